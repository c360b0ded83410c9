/*
 * sanitize_driver.c -- runs every entry point of the CPU oracle on seeded
 * small inputs so that a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer can watch each memory access and arithmetic operation (test
 * infrastructure: the CPU suite compiles and runs it; nothing else uses it).
 *
 * Inputs cover the cases with boundary arithmetic: rays that miss the map or
 * run parallel to its faces, cameras inside occupied voxels and outside the
 * map, 1x1 / 1xH / Wx1 endpoint grids, one-voxel and non-cubic maps,
 * non-finite poses, trajectories whose voxel box is the whole map, and depth
 * images with dropped pixels, returns beyond the range and returns outside
 * the map.  The exit status is non-zero when a result breaks an invariant
 * that holds for any input (steps <= nx+ny+nz+3, union counts add up).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nbt_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ULL;

/* splitmix64 (Steele, Lea and Flood 2014) */
static uint64_t next_u64(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static double uniform(double lo, double hi) { return lo + (hi - lo) * (double)(next_u64() >> 11) * 0x1p-53; }

/* Row-major camera->world rotation with z towards (tx,ty,tz) - p, x horizontal. */
static void look_at(const double p[3], const double q[3], float pose[12])
{
    double z[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double nz = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    if (nz == 0.0) { z[0] = 0; z[1] = 0; z[2] = -1; nz = 1; }
    for (int a = 0; a < 3; ++a) z[a] /= nz;
    double up[3] = {0, 0, 1};
    if (fabs(z[2]) > 0.9999) { up[1] = 1; up[2] = 0; }
    double x[3] = {z[1] * up[2] - z[2] * up[1], z[2] * up[0] - z[0] * up[2], z[0] * up[1] - z[1] * up[0]};
    const double nx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int a = 0; a < 3; ++a) x[a] /= nx;
    const double y[3] = {z[1] * x[2] - z[2] * x[1], z[2] * x[0] - z[0] * x[2], z[0] * x[1] - z[1] * x[0]};
    for (int a = 0; a < 3; ++a) {
        pose[3 * a + 0] = (float)x[a];
        pose[3 * a + 1] = (float)y[a];
        pose[3 * a + 2] = (float)z[a];
        pose[9 + a] = (float)p[a];
    }
}

static int failures = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            fprintf(stderr, __VA_ARGS__);     \
            fputc('\n', stderr);              \
            ++failures;                       \
        }                                     \
    } while (0)

static void run_map(int nx, int ny, int nz, float voxel, int n_poses, int W, int H, int traj_len)
{
    const int64_t nvox = (int64_t)nx * ny * nz;
    float* P = malloc(sizeof(float) * nvox);
    const float vals[4] = {0.2f, 0.5f, 0.9f, 0.0f};
    for (int64_t k = 0; k < nvox; ++k) P[k] = vals[next_u64() % 4];
    oracle_map m = {P, nx, ny, nz, voxel, {-0.1f, 0.05f, 0.2f}, 0.5f, 0.5f};
    oracle_camera cam = {W, H, 0.57735f, 0.41421f, 1.2f * voxel * (float)(nx + ny + nz)};
    const double c[3] = {m.origin[0] + 0.5 * nx * voxel, m.origin[1] + 0.5 * ny * voxel,
                         m.origin[2] + 0.5 * nz * voxel};
    const double ext = voxel * (double)(nx + ny + nz);

    float* poses = malloc(sizeof(float) * 12 * n_poses);
    for (int p = 0; p < n_poses; ++p) {
        double pos[3], tgt[3] = {c[0], c[1], c[2]};
        for (int a = 0; a < 3; ++a) pos[a] = c[a] + uniform(-1.0, 1.0) * ext;
        if (p % 7 == 1) for (int a = 0; a < 3; ++a) tgt[a] = pos[a] + (a == p % 3 ? 1.0 : 0.0); /* axis-parallel */
        if (p % 7 == 2) for (int a = 0; a < 3; ++a) tgt[a] = 2 * pos[a] - c[a];                 /* looks away */
        if (p % 7 == 3) for (int a = 0; a < 3; ++a) pos[a] = c[a];                              /* inside */
        look_at(pos, tgt, poses + 12 * p);
        if (p % 11 == 5) poses[12 * p + 9 + p % 3] = NAN;                                      /* invalid */
    }

    const int64_t rays = (int64_t)W * H;
    uint32_t* steps = malloc(sizeof(uint32_t) * rays * n_poses);
    int32_t* stop = malloc(sizeof(int32_t) * rays * n_poses);
    int32_t* reason = malloc(sizeof(int32_t) * rays * n_poses);
    uint64_t* hash = malloc(sizeof(uint64_t) * rays * n_poses);
    double* gain = malloc(sizeof(double) * rays * n_poses);
    oracle_trace_rays(&m, &cam, poses, n_poses, steps, stop, reason, hash, gain);
    for (int64_t r = 0; r < rays * n_poses; ++r) {
        CHECK(steps[r] <= (uint32_t)(nx + ny + nz + 3), "ray %lld: %u steps", (long long)r, steps[r]);
        CHECK(stop[r] >= -1 && stop[r] < nvox, "ray %lld: stop %d", (long long)r, stop[r]);
        CHECK(reason[r] >= ORACLE_MISS && reason[r] <= ORACLE_INVALID, "ray %lld: reason", (long long)r);
    }

    const int cap = nx + ny + nz + 3;
    int32_t* path = malloc(sizeof(int32_t) * cap);
    for (int p = 0; p < n_poses; ++p) {
        oracle_ray ray;
        oracle_cast_ray(&m, &cam, poses + 12 * p, W - 1, 0, path, cap, &ray);
        oracle_cast_ray(&m, &cam, poses + 12 * p, 0, H - 1, NULL, 0, &ray);
        oracle_cast_ray(&m, &cam, poses + 12 * p, W / 2, H / 2, path, 2, &ray);   /* short path buffer */
    }

    float* ig = malloc(sizeof(float) * n_poses);
    uint64_t* st = malloc(sizeof(uint64_t) * n_poses);
    oracle_eval_viewpoints(&m, &cam, poses, n_poses, ig, st);

    if (traj_len > 0 && n_poses >= traj_len) {
        const int64_t T = n_poses / traj_len;
        float* igu = malloc(sizeof(float) * T);
        uint32_t* cnt = malloc(sizeof(uint32_t) * 4 * T);
        uint64_t* vis = malloc(sizeof(uint64_t) * T);
        CHECK(oracle_eval_trajectories(&m, &cam, poses, T, traj_len, igu, cnt, vis) == 0, "trajectories");
        for (int64_t t = 0; t < T; ++t) {
            CHECK(cnt[4 * t] == cnt[4 * t + 1] + cnt[4 * t + 2] + cnt[4 * t + 3], "traj %lld counts", (long long)t);
            CHECK((int64_t)cnt[4 * t] <= nvox, "traj %lld: more voxels than the map", (long long)t);
        }
        free(igu); free(cnt); free(vis);
    }

    /* depth insertion: z-depths around the map, some dropped, some beyond range */
    float* depth = malloc(sizeof(float) * rays * n_poses);
    for (int64_t r = 0; r < rays * n_poses; ++r) {
        const uint64_t k = next_u64() % 8;
        depth[r] = k == 0 ? 0.0f : k == 1 ? NAN : k == 2 ? 2.0f * cam.range : k == 3 ? cam.range
                                                                                    : (float)uniform(0.0, 1.5 * ext);
    }
    float* L = calloc((size_t)nvox, sizeof(float));
    CHECK(oracle_insert_scans(&m, &cam, poses, depth, n_poses, 0.85f, -0.4f, -2.0f, 3.5f, L) == 0, "insert");
    for (int64_t k = 0; k < nvox; ++k) CHECK(L[k] >= -2.0f && L[k] <= 3.5f, "log-odds %lld out of bounds", (long long)k);

    free(L); free(depth); free(ig); free(st); free(path);
    free(steps); free(stop); free(reason); free(hash); free(gain);
    free(poses); free(P);
}

int main(void)
{
    const uint8_t abc[3] = {'a', 'b', 'c'};
    CHECK(oracle_fnv1a_bytes(abc, 0) == 0xcbf29ce484222325ULL, "fnv basis");
    CHECK(oracle_fnv1a_bytes(abc, 1) == 0xaf63dc4c8601ec8cULL, "fnv 'a'");
    run_map(1, 1, 1, 0.5f, 14, 3, 2, 7);
    run_map(12, 9, 7, 0.1f, 22, 7, 5, 11);
    run_map(16, 16, 16, 0.05f, 33, 1, 1, 3);
    run_map(5, 23, 3, 0.2f, 12, 1, 9, 4);
    run_map(31, 2, 17, 0.07f, 18, 13, 1, 6);
    run_map(24, 20, 28, 0.04f, 24, 16, 12, 8);
    if (failures) {
        fprintf(stderr, "%d invariant failures\n", failures);
        return 1;
    }
    printf("oracle sanitize driver ok\n");
    return 0;
}
