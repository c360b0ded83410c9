/*
 * nbt_oracle.c -- CPU oracle for information-gain raycasting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, includes or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it, to check and to time the GPU path.  It is written
 * for a reader holding the paper, in the most direct form possible: single
 * thread, one ray at a time, one voxel at a time, no blocking or reordering.
 *
 * What it computes (Renz et al., "Next-Best-Trajectory Planning of Robot
 * Manipulators for Effective Observation and Exploration", Sec. III):
 *   - Endpoint calculation: a W x H grid of endpoints on the far frustum
 *     plane at depth d_Cam, bounded by the border rays at
 *     d_h = d_Cam tan(FoV_h/2) and d_v = d_Cam tan(FoV_v/2).
 *   - IG calculation: for every ray from the perspective to an endpoint,
 *     g_R = sum of g(v_i) over the encountered voxels up to and including
 *     the first occupied one, or up to the endpoint (Eq. 2 and the N_O
 *     stop rule), and g_P = mean of g_R over the N_E = W*H rays.
 *   - Voxel states from probabilities: Occupied if P > occ_threshold, Free if
 *     P < free_threshold, Unknown otherwise; g = 1-P, P, 1 (Eq. 2).
 * The traversal itself is not named in the paper; this oracle walks the
 * voxels with the incremental grid traversal of Amanatides and Woo
 * ("A Fast Voxel Traversal Algorithm for Ray Tracing", Eurographics 1987),
 * with the conventions fixed below.
 *
 * Floating point: every ray-geometry quantity is an IEEE binary32 value and
 * each operation below is a single rounded binary32 operation (the file is
 * compiled with -ffp-contract=off and without fast-math, so no fused
 * multiply-add is formed).  Gains are accumulated in binary64.
 *
 * Conventions fixed here (the paper is silent on them):
 *   C1  Ray k = j*W + i, i along the camera x axis, j along its y axis.
 *       Endpoint in camera coordinates (u, v, d_Cam) with
 *       u = d_h * ((2i-(W-1)) / (W-1))  (u = 0 when W == 1), likewise v.
 *       The grid includes the border (corner) rays.
 *   C2  Pose = row-major R (camera->world) then t.  World endpoint
 *       e = t + ((R0*u + R1*v) + R2*d_Cam) per row.
 *   C3  Voxel coordinates: O = (t - origin)*inv_s, E = (e - origin)*inv_s,
 *       D = E - O, inv_s = 1/s_Vox.
 *   C4  The segment is clipped to the map box [0, n) per axis and to
 *       parameter range [0, 1]; voxels outside the map do not exist.  An
 *       axis with |D| < 2^-100 is treated as parallel to the faces.
 *   C5  Start voxel: floor(O + t0*D), clamped into the map.
 *   C6  Each step visits the current voxel first; then the axis with the
 *       smallest crossing parameter advances (ties go to the lower axis:
 *       x before y before z).  If that crossing lies beyond t1 the ray
 *       ends (END when the endpoint was inside the map, EXIT otherwise);
 *       a crossing exactly at t1 still advances.  Advancing out of the map
 *       also ends the ray (EXIT).
 *   C7  A ray whose voxel coordinates are not all finite is INVALID; it
 *       visits nothing and makes its perspective's IG NaN.
 *   C8  Trajectory union: the set of voxels visited by any ray of any pose
 *       of the trajectory; each counts once.
 *
 * Map update by depth-image insertion (the occupancy update that precedes
 * IG evaluation, Sec. II-III: the map is built from the camera's point
 * clouds; the paper delegates it to UfoMap and gives no formulas, so the
 * standard log-odds occupancy update with clamping is written out here):
 *   I1  Scan k = a pose plus a W x H depth image; D[j][i] is the z-depth in
 *       metres of the return along pixel (i, j)'s ray of C1-C3 (that ray's
 *       endpoint lies at z-depth d_Cam), so the return sits at segment
 *       parameter s = D / d_Cam (one binary32 division).
 *   I2  D not a number or D <= 0: no measurement, the ray is skipped.
 *       s >= 1 (D = +inf included): no return within range; the segment
 *       [0, 1] is carved free and nothing is hit.
 *   I3  Otherwise the segment is [0, s]: the walk of C4-C6 with t1 replaced
 *       by min(t1, s) and without the occupied stop.  If s <= t1 (the return
 *       lies inside the map) the last voxel of the walk is hit and the
 *       others are free; otherwise every voxel of the walk is free.
 *   I4  Per scan (discrete insertion): H = voxels hit by any ray, F = voxels
 *       free for any ray and not in H.  Each log-odds value L is updated
 *       once per scan: L + l_hit on H, L + l_miss on F, then clamped as
 *       min(max(L', l_min), l_max), all in binary32; other voxels keep L.
 *   I5  Scans are applied in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "nbt_oracle.h"

/* ---- small helpers, written out so every comparison is explicit ---- */

static float sel_min(float a, float b) { return (b < a) ? b : a; }
static float sel_max(float a, float b) { return (b > a) ? b : a; }

static int is_finite_f(float x) { return x == x && x - x == 0.0f; }

/* FNV-1a, 64-bit (Fowler, Noll, Vo): xor each byte, then multiply. */
static uint64_t fnv1a_u32(uint64_t h, int32_t value)
{
    uint32_t u = (uint32_t)value;
    for (int b = 0; b < 4; ++b) {
        h ^= (uint64_t)((u >> (8 * b)) & 0xFFu);
        h *= 0x100000001b3ULL;
    }
    return h;
}

uint64_t oracle_fnv1a_bytes(const uint8_t* bytes, int64_t n)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int64_t k = 0; k < n; ++k) {
        h ^= (uint64_t)bytes[k];
        h *= 0x100000001b3ULL;
    }
    return h;
}

/* Eq. 2: the information gain of one voxel from its probability. */
static double voxel_gain(const oracle_map* m, float p, int* state)
{
    if (p > m->occ_threshold) {
        *state = ORACLE_OCCUPIED;
        return (double)(1.0f - p);
    }
    if (p < m->free_threshold) {
        *state = ORACLE_FREE;
        return (double)p;
    }
    *state = ORACLE_UNKNOWN;
    return 1.0;
}

/*
 * Cast ray (i, j) of one perspective.  Fills *out; if path != NULL the linear
 * indices of the visited voxels are written there (capacity path_cap; the
 * count written is min(steps, path_cap)).
 */
void oracle_cast_ray(const oracle_map* m, const oracle_camera* cam, const float* pose,
                     int i, int j, int32_t* path, int path_cap, oracle_ray* out)
{
    const int n[3] = {m->nx, m->ny, m->nz};
    out->steps = 0;
    out->stop_lin = -1;
    out->reason = ORACLE_MISS;
    out->hash = 0xcbf29ce484222325ULL;
    out->gain = 0.0;

    /* far-plane half extents and inverse voxel size */
    const float dh = cam->range * cam->tan_half_h;
    const float dv = cam->range * cam->tan_half_v;
    const float inv_s = 1.0f / m->voxel;

    /* C1: endpoint in camera coordinates */
    float u = 0.0f, v = 0.0f;
    if (cam->width > 1)
        u = dh * ((float)(2 * i - (cam->width - 1)) / (float)(cam->width - 1));
    if (cam->height > 1)
        v = dv * ((float)(2 * j - (cam->height - 1)) / (float)(cam->height - 1));
    const float c[3] = {u, v, cam->range};

    /* C2, C3: world endpoint and voxel-unit segment O -> E */
    float O[3], E[3], D[3];
    for (int a = 0; a < 3; ++a) {
        const float* row = pose + 3 * a;
        float w = row[0] * c[0];
        w = w + row[1] * c[1];
        w = w + row[2] * c[2];
        const float t = pose[9 + a];
        const float e = t + w;
        O[a] = (t - m->origin[a]) * inv_s;
        E[a] = (e - m->origin[a]) * inv_s;
        D[a] = E[a] - O[a];
    }
    for (int a = 0; a < 3; ++a) {
        if (!is_finite_f(O[a]) || !is_finite_f(E[a]) || !is_finite_f(D[a])) {
            out->reason = ORACLE_INVALID;
            out->gain = NAN;
            return;
        }
    }

    /* C4: clip to the map box and to [0, 1] */
    float t0 = 0.0f, t1 = 1.0f;
    float inv[3];
    int parallel[3];
    for (int a = 0; a < 3; ++a) {
        parallel[a] = fabsf(D[a]) < 0x1p-100f;
        if (parallel[a]) {
            if (!(O[a] >= 0.0f && O[a] < (float)n[a]))
                return; /* MISS: runs beside the map */
            inv[a] = 0.0f;
            continue;
        }
        inv[a] = 1.0f / D[a];
        const float tA = (0.0f - O[a]) * inv[a];
        const float tB = ((float)n[a] - O[a]) * inv[a];
        t0 = sel_max(t0, sel_min(tA, tB));
        t1 = sel_min(t1, sel_max(tA, tB));
    }
    if (t0 > t1)
        return; /* MISS */

    /* C5: start voxel; C6 set-up */
    int idx[3], step[3];
    float tmax[3], tdelta[3];
    for (int a = 0; a < 3; ++a) {
        float f = floorf(O[a] + t0 * D[a]);
        f = sel_max(f, 0.0f);
        f = sel_min(f, (float)(n[a] - 1));
        idx[a] = (int)f;
        if (parallel[a]) {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdelta[a] = INFINITY;
        } else {
            step[a] = D[a] > 0.0f ? 1 : -1;
            tdelta[a] = fabsf(inv[a]);
            tmax[a] = ((float)(idx[a] + (step[a] > 0 ? 1 : 0)) - O[a]) * inv[a];
        }
    }

    /* C6: visit voxels until the first occupied one, the end or the map edge */
    const int guard = m->nx + m->ny + m->nz + 3;
    uint64_t h = 0xcbf29ce484222325ULL;
    double acc = 0.0;
    uint32_t steps = 0;
    int32_t lin = -1;
    int reason = ORACLE_EXIT;
    while ((int)steps < guard) {
        lin = (idx[2] * m->ny + idx[1]) * m->nx + idx[0];
        if (path != NULL && (int)steps < path_cap)
            path[steps] = lin;
        steps += 1;
        h = fnv1a_u32(h, lin);
        int state;
        acc += voxel_gain(m, m->P[lin], &state);
        if (state == ORACLE_OCCUPIED) {
            reason = ORACLE_HIT;
            break;
        }
        int a;
        if (tmax[0] <= tmax[1] && tmax[0] <= tmax[2])
            a = 0;
        else if (tmax[1] <= tmax[2])
            a = 1;
        else
            a = 2;
        if (tmax[a] > t1) {
            reason = (t1 == 1.0f) ? ORACLE_END : ORACLE_EXIT;
            break;
        }
        idx[a] += step[a];
        if (idx[a] < 0 || idx[a] >= n[a]) {
            reason = ORACLE_EXIT;
            break;
        }
        tmax[a] = tmax[a] + tdelta[a];
    }
    out->steps = steps;
    out->stop_lin = lin;
    out->reason = reason;
    out->hash = h;
    out->gain = acc;
}

void oracle_trace_rays(const oracle_map* m, const oracle_camera* cam, const float* poses,
                       int64_t n_poses, uint32_t* steps, int32_t* stop_lin, int32_t* reason,
                       uint64_t* hash, double* gain)
{
    const int64_t rays = (int64_t)cam->width * cam->height;
    for (int64_t p = 0; p < n_poses; ++p) {
        for (int j = 0; j < cam->height; ++j) {
            for (int i = 0; i < cam->width; ++i) {
                oracle_ray r;
                oracle_cast_ray(m, cam, poses + 12 * p, i, j, NULL, 0, &r);
                const int64_t k = p * rays + (int64_t)j * cam->width + i;
                steps[k] = r.steps;
                stop_lin[k] = r.stop_lin;
                reason[k] = r.reason;
                hash[k] = r.hash;
                gain[k] = r.gain;
            }
        }
    }
}

/* g_P = (1/N_E) sum_k g_R,k for every perspective. */
void oracle_eval_viewpoints(const oracle_map* m, const oracle_camera* cam, const float* poses,
                            int64_t n_poses, float* ig_out, uint64_t* steps_out)
{
    const int64_t rays = (int64_t)cam->width * cam->height;
    for (int64_t p = 0; p < n_poses; ++p) {
        double sum = 0.0;
        uint64_t st = 0;
        for (int j = 0; j < cam->height; ++j) {
            for (int i = 0; i < cam->width; ++i) {
                oracle_ray r;
                oracle_cast_ray(m, cam, poses + 12 * p, i, j, NULL, 0, &r);
                sum += r.gain;
                st += r.steps;
            }
        }
        ig_out[p] = (float)(sum / (double)rays);
        if (steps_out != NULL)
            steps_out[p] = st;
    }
}

/*
 * Trajectory union (C8): every voxel visited by any ray of any of the L poses
 * counts once.  counts[4*t + {0,1,2,3}] = |U|, occupied, free, unknown;
 * visits[t] = total voxel visits (sum of ray steps); ig_union[t] = sum of the
 * gains of the voxels in U (binary64, rounded once), NaN if any ray of the
 * trajectory is INVALID (C7).
 */
int oracle_eval_trajectories(const oracle_map* m, const oracle_camera* cam, const float* poses,
                             int64_t n_traj, int64_t poses_per_traj, float* ig_union,
                             uint32_t* counts, uint64_t* visits)
{
    const int64_t nvox = (int64_t)m->nx * m->ny * m->nz;
    const int cap = m->nx + m->ny + m->nz + 3;
    uint8_t* seen = (uint8_t*)calloc((size_t)nvox, 1);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t list_cap = 1 << 16, list_n = 0;
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)list_cap);
    if (!seen || !path || !list) {
        free(seen); free(path); free(list);
        return -1;
    }
    for (int64_t t = 0; t < n_traj; ++t) {
        uint64_t total = 0;
        int invalid = 0;
        list_n = 0;
        for (int64_t l = 0; l < poses_per_traj; ++l) {
            const float* pose = poses + 12 * (t * poses_per_traj + l);
            for (int j = 0; j < cam->height; ++j) {
                for (int i = 0; i < cam->width; ++i) {
                    oracle_ray r;
                    oracle_cast_ray(m, cam, pose, i, j, path, cap, &r);
                    total += r.steps;
                    if (r.reason == ORACLE_INVALID)
                        invalid = 1;
                    for (uint32_t s = 0; s < r.steps; ++s) {
                        const int32_t v = path[s];
                        if (!seen[v]) {
                            seen[v] = 1;
                            if (list_n == list_cap) {
                                list_cap *= 2;
                                int32_t* grown = (int32_t*)realloc(list, sizeof(int32_t) * (size_t)list_cap);
                                if (!grown) {
                                    free(seen); free(path); free(list);
                                    return -1;
                                }
                                list = grown;
                            }
                            list[list_n++] = v;
                        }
                    }
                }
            }
        }
        uint32_t c_occ = 0, c_free = 0, c_unk = 0;
        double g = 0.0;
        for (int64_t q = 0; q < list_n; ++q) {
            int state;
            g += voxel_gain(m, m->P[list[q]], &state);
            if (state == ORACLE_OCCUPIED) c_occ++;
            else if (state == ORACLE_FREE) c_free++;
            else c_unk++;
            seen[list[q]] = 0;
        }
        counts[4 * t + 0] = (uint32_t)list_n;
        counts[4 * t + 1] = c_occ;
        counts[4 * t + 2] = c_free;
        counts[4 * t + 3] = c_unk;
        visits[t] = total;
        ig_union[t] = invalid ? NAN : (float)g;
    }
    free(seen);
    free(path);
    free(list);
    return 0;
}

/*
 * Log-odds occupancy update from depth images (I1-I5).  Only the geometry
 * of *m is used (not m->P).  logodds: [nz][ny][nx], updated in place.
 * Returns 0, or -1 when out of memory.
 */
int oracle_insert_scans(const oracle_map* m, const oracle_camera* cam, const float* poses,
                        const float* depth, int64_t n_scans, float l_hit, float l_miss,
                        float l_min, float l_max, float* logodds)
{
    enum { MARK_FREE = 1, MARK_HIT = 2 };
    const int n[3] = {m->nx, m->ny, m->nz};
    const int64_t nvox = (int64_t)m->nx * m->ny * m->nz;
    uint8_t* mark = (uint8_t*)calloc((size_t)(nvox > 0 ? nvox : 1), 1);
    if (!mark)
        return -1;
    const float dh = cam->range * cam->tan_half_h;
    const float dv = cam->range * cam->tan_half_v;
    const float inv_s = 1.0f / m->voxel;
    const int guard = m->nx + m->ny + m->nz + 3;

    for (int64_t k = 0; k < n_scans; ++k) {
        const float* pose = poses + 12 * k;
        const float* img = depth + k * (int64_t)cam->width * cam->height;
        for (int j = 0; j < cam->height; ++j) {
            for (int i = 0; i < cam->width; ++i) {
                /* I1, I2: the measurement and the segment end */
                const float d = img[(int64_t)j * cam->width + i];
                if (!(d > 0.0f))
                    continue; /* no measurement (NaN fails the test too) */
                const float s = d / cam->range;
                const int ret = s < 1.0f; /* a return within range */

                /* C1-C3: the pixel's ray, as in oracle_cast_ray */
                float u = 0.0f, v = 0.0f;
                if (cam->width > 1)
                    u = dh * ((float)(2 * i - (cam->width - 1)) / (float)(cam->width - 1));
                if (cam->height > 1)
                    v = dv * ((float)(2 * j - (cam->height - 1)) / (float)(cam->height - 1));
                const float c[3] = {u, v, cam->range};
                float O[3], E[3], D[3];
                int finite = 1;
                for (int a = 0; a < 3; ++a) {
                    const float* row = pose + 3 * a;
                    float w = row[0] * c[0];
                    w = w + row[1] * c[1];
                    w = w + row[2] * c[2];
                    const float t = pose[9 + a];
                    const float e = t + w;
                    O[a] = (t - m->origin[a]) * inv_s;
                    E[a] = (e - m->origin[a]) * inv_s;
                    D[a] = E[a] - O[a];
                    finite = finite && is_finite_f(O[a]) && is_finite_f(E[a]) && is_finite_f(D[a]);
                }
                if (!finite)
                    continue; /* C7: an invalid ray updates nothing */

                /* C4: clip to the map box and to [0, 1] */
                float t0 = 0.0f, t1 = 1.0f;
                float inv[3];
                int parallel[3], miss = 0;
                for (int a = 0; a < 3; ++a) {
                    parallel[a] = fabsf(D[a]) < 0x1p-100f;
                    if (parallel[a]) {
                        if (!(O[a] >= 0.0f && O[a] < (float)n[a]))
                            miss = 1;
                        inv[a] = 0.0f;
                        continue;
                    }
                    inv[a] = 1.0f / D[a];
                    const float tA = (0.0f - O[a]) * inv[a];
                    const float tB = ((float)n[a] - O[a]) * inv[a];
                    t0 = sel_max(t0, sel_min(tA, tB));
                    t1 = sel_min(t1, sel_max(tA, tB));
                }
                /* I3: the segment ends at the return when there is one */
                const int inside = ret && s <= t1;
                if (ret)
                    t1 = sel_min(t1, s);
                if (miss || t0 > t1)
                    continue;

                /* C5 */
                int idx[3], step[3];
                float tmax[3], tdelta[3];
                for (int a = 0; a < 3; ++a) {
                    float f = floorf(O[a] + t0 * D[a]);
                    f = sel_max(f, 0.0f);
                    f = sel_min(f, (float)(n[a] - 1));
                    idx[a] = (int)f;
                    if (parallel[a]) {
                        step[a] = 0;
                        tmax[a] = INFINITY;
                        tdelta[a] = INFINITY;
                    } else {
                        step[a] = D[a] > 0.0f ? 1 : -1;
                        tdelta[a] = fabsf(inv[a]);
                        tmax[a] = ((float)(idx[a] + (step[a] > 0 ? 1 : 0)) - O[a]) * inv[a];
                    }
                }

                /* C6 without the occupied stop; the last voxel is hit if I3 says so */
                for (int visited = 0; visited < guard; ++visited) {
                    const int64_t lin = ((int64_t)idx[2] * m->ny + idx[1]) * m->nx + idx[0];
                    int a;
                    if (tmax[0] <= tmax[1] && tmax[0] <= tmax[2])
                        a = 0;
                    else if (tmax[1] <= tmax[2])
                        a = 1;
                    else
                        a = 2;
                    if (tmax[a] > t1) {
                        mark[lin] |= inside ? MARK_HIT : MARK_FREE;
                        break;
                    }
                    mark[lin] |= MARK_FREE;
                    idx[a] += step[a];
                    if (idx[a] < 0 || idx[a] >= n[a])
                        break;
                    tmax[a] = tmax[a] + tdelta[a];
                }
            }
        }
        /* I4: one update per marked voxel, hit before free */
        for (int64_t q = 0; q < nvox; ++q) {
            if (!mark[q])
                continue;
            float l = logodds[q] + ((mark[q] & MARK_HIT) ? l_hit : l_miss);
            l = sel_max(l, l_min);
            l = sel_min(l, l_max);
            logodds[q] = l;
            mark[q] = 0;
        }
    }
    free(mark);
    return 0;
}
