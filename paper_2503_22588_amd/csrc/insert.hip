// insert.hip -- map update by depth-image insertion (clamped log-odds occupancy update).
//
// The step before IG evaluation: the map is built from the camera's point
// clouds (Sec. II-III; the paper leaves the update to its occupancy-mapping
// library and gives no formulas).  Per scan (a pose and a W x H z-depth
// image):
//   - the return of pixel (i, j) lies on that pixel's endpoint ray (Sec. III,
//     endpoint calculation; the endpoint sits at z-depth d_Cam) at segment
//     parameter s = depth / d_Cam;
//   - depth NaN or <= 0: no measurement; s >= 1: no return within range, the
//     whole segment is carved free;
//   - the walk is the ray walk of the IG kernels (same set-up and stepping,
//     ties to the lower axis) ending at min(t1, s) and not stopping at
//     occupied voxels; its last voxel is hit when the return lies inside the
//     map, every other voxel it visits is free;
//   - each voxel marked in the scan moves once: log-odds + l_hit if any ray
//     hit it, else + l_miss, then clamped to [l_min, l_max] (binary32).
// Scans are applied in order.  Two passes per scan: a mark pass (one thread
// per pixel; two mark bytes per voxel, pass and return, each set by a plain
// byte store on every visit) and an apply pass (one thread per 2
// voxels: it reads their marks, updates the marked log-odds values and
// clears the marks for the next scan).
#include "host.hpp"
#include "ray.hpp"

namespace nbt {

// Two mark bytes per voxel, set by plain byte stores (a byte store touches
// no neighbouring byte, and any number of rays may store the same 1):
// byte 2v says a ray passed voxel v, byte 2v + 1 that a ray's return lies in it.
constexpr uint32_t kMarkFree = 0u, kMarkHit = 1u;

// Every visit stores its mark.  Checking first (a load, then a store only
// where the mark is unset) saves stores on the voxels near the camera that
// all rays pass, but puts a load's latency on every step: slower.
__device__ __forceinline__ void mark_voxel(uint8_t* marks, uint32_t lin, uint32_t kind) {
    marks[2 * (size_t)lin + kind] = 1;
}

__global__ __launch_bounds__(256) void insert_mark_kernel(DevMap m, CamParams c,
                                                          const float* __restrict__ pose_in,
                                                          const float* __restrict__ depth,
                                                          uint8_t* __restrict__ marks) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (uint32_t)c.W * (uint32_t)c.H) return;
    const int i = (int)(k % (uint32_t)c.W), j = (int)(k / (uint32_t)c.W);
    const float d = depth[k];
    if (!(d > 0.0f)) return;                 // no measurement (NaN included)
    const float s = d / c.range;
    const bool ret = s < 1.0f;               // a return within range

    // the pixel's segment O -> E in voxel units, as in setup_ray
    float u = 0.0f, v = 0.0f;
    if (c.W > 1) u = c.dh * ((float)(2 * i - (c.W - 1)) / (float)(c.W - 1));
    if (c.H > 1) v = c.dv * ((float)(2 * j - (c.H - 1)) / (float)(c.H - 1));
    const float org[3] = {m.ox, m.oy, m.oz};
    float O[3], D[3];
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float w = pose_in[3 * a + 0] * u;
        w = w + pose_in[3 * a + 1] * v;
        w = w + pose_in[3 * a + 2] * c.range;
        const float t = pose_in[9 + a];
        const float e = t + w;
        O[a] = (t - org[a]) * m.inv_s;
        const float E = (e - org[a]) * m.inv_s;
        D[a] = E - O[a];
        finite = finite && __builtin_isfinite(O[a]) && __builtin_isfinite(E) && __builtin_isfinite(D[a]);
    }
    if (!finite) return;                     // an invalid ray updates nothing

    float t0 = 0.0f, t1 = 1.0f;
    float inv[3];
    bool par[3];
    const int n[3] = {m.nx, m.ny, m.nz};
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = clip_axis(O[a], D[a], n[a], t0, t1, inv[a], par[a]) && inside;
    const bool hit_inside = ret && s <= t1;  // the return lies inside the map
    if (ret) t1 = sel_min(t1, s);
    if (!inside || t0 > t1) return;

    int ix, iy, iz, sx, sy, sz;
    float tx, ty, tz, dtx, dty, dtz;
    init_axis(O[0], D[0], t0, inv[0], par[0], n[0], ix, sx, tx, dtx);
    init_axis(O[1], D[1], t0, inv[1], par[1], n[1], iy, sy, ty, dty);
    init_axis(O[2], D[2], t0, inv[2], par[2], n[2], iz, sz, tz, dtz);

    const int guard = m.nx + m.ny + m.nz + 3;
    for (int visited = 0; visited < guard; ++visited) {
        const uint32_t lin = ((uint32_t)iz * (uint32_t)m.ny + (uint32_t)iy) * (uint32_t)m.nx + (uint32_t)ix;
        const bool ax = tx <= ty && tx <= tz;
        const bool ay = !ax && ty <= tz;
        const float tn = ax ? tx : (ay ? ty : tz);
        if (tn > t1) {
            mark_voxel(marks, lin, hit_inside ? kMarkHit : kMarkFree);
            break;
        }
        mark_voxel(marks, lin, kMarkFree);
        if (ax) {
            ix += sx;
            if ((uint32_t)ix >= (uint32_t)m.nx) break;
            tx = tx + dtx;
        } else if (ay) {
            iy += sy;
            if ((uint32_t)iy >= (uint32_t)m.ny) break;
            ty = ty + dty;
        } else {
            iz += sz;
            if ((uint32_t)iz >= (uint32_t)m.nz) break;
            tz = tz + dtz;
        }
    }
}

__global__ __launch_bounds__(256) void insert_apply_kernel(uint32_t* __restrict__ marks,
                                                           float* __restrict__ L, uint64_t nvox,
                                                           nbt_ig_insert_params p) {
    // one thread per mark word: two voxels, (pass, return) bytes each
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= (nvox + 1) / 2) return;
    const uint32_t mk = marks[w];
    if (mk == 0u) return;
    marks[w] = 0u;
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b) {
        const uint64_t v = 2 * w + b;
        const uint32_t pass = (mk >> (16u * b)) & 0xFFu, hit = (mk >> (16u * b + 8u)) & 0xFFu;
        if ((pass | hit) == 0u || v >= nvox) continue;
        float l = L[v] + (hit ? p.l_hit : p.l_miss);
        l = (p.l_min > l) ? p.l_min : l;
        l = (p.l_max < l) ? p.l_max : l;
        L[v] = l;
    }
}

__global__ __launch_bounds__(256) void logodds_to_prob_kernel(const float* __restrict__ L,
                                                              float* __restrict__ P, uint64_t nvox) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    P[v] = 1.0f / (1.0f + expf(-L[v]));
}

}  // namespace nbt

using namespace nbt;

extern "C" uint64_t nbt_ig_insert_workspace_words(const nbt_ig_map* map) {
    if (!map) return 0;
    return ((uint64_t)map->dm.nx * (uint64_t)map->dm.ny * (uint64_t)map->dm.nz + 1) / 2;
}

extern "C" nbt_ig_insert_params nbt_ig_insert_default_params(void) {
    // log(p / (1 - p)) for hit 0.7, miss 0.4 and the bounds 0.1192 and 0.971, in binary32
    return nbt_ig_insert_params{0x1.b1d106p-1f, -0x1.9f323ep-2f, -0x1.0000eap+1f, 0x1.c16974p+1f};
}

extern "C" int nbt_ig_insert_scans(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                   const float* depth, uint32_t n_scans, const nbt_ig_insert_params* params,
                                   float* logodds, float* prob_out, uint32_t* workspace,
                                   uint64_t workspace_words, void* stream) {
    if (int rc = check_map(map)) return rc;
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    if (!logodds || !workspace) return fail(NBT_IG_EINVAL, "logodds or workspace is NULL");
    if (workspace_words < nbt_ig_insert_workspace_words(map))
        return fail(NBT_IG_EINVAL, "workspace holds %llu words, the map needs %llu",
                    (unsigned long long)workspace_words,
                    (unsigned long long)nbt_ig_insert_workspace_words(map));
    if (n_scans > 0 && (!poses || !depth)) return fail(NBT_IG_EINVAL, "poses or depth is NULL");
    const nbt_ig_insert_params p = params ? *params : nbt_ig_insert_default_params();
    if (!std::isfinite(p.l_hit) || !std::isfinite(p.l_miss) || !std::isfinite(p.l_min) ||
        !std::isfinite(p.l_max) || !(p.l_min <= p.l_max))
        return fail(NBT_IG_EINVAL, "insertion parameters must be finite with l_min <= l_max");
    const uint64_t rays = (uint64_t)c.W * (uint64_t)c.H;
    const uint64_t nvox = (uint64_t)map->dm.nx * (uint64_t)map->dm.ny * (uint64_t)map->dm.nz;
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const unsigned mark_blocks = (unsigned)((rays + 255) / 256);
    const unsigned apply_blocks = (unsigned)(((nvox + 1) / 2 + 255) / 256);
    for (uint32_t k = 0; k < n_scans; ++k) {
        hipLaunchKernelGGL(insert_mark_kernel, dim3(mark_blocks), dim3(256), 0, s, map->dm, c,
                           poses + 12 * (size_t)k, depth + rays * k, reinterpret_cast<uint8_t*>(workspace));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "insert_mark_kernel");
        hipLaunchKernelGGL(insert_apply_kernel, dim3(apply_blocks), dim3(256), 0, s, workspace, logodds, nvox, p);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "insert_apply_kernel");
    }
    if (prob_out) {
        hipLaunchKernelGGL(logodds_to_prob_kernel, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, s,
                           logodds, prob_out, nvox);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "logodds_to_prob_kernel");
    }
    return NBT_IG_OK;
}
