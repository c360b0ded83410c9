// raycast_viewpoints.hip -- per-perspective IG and the parity-mode ray records.
//
// Work decomposition: a perspective's N_E rays are cut into pixel tiles of
// 64 rays, one tile per wavefront (one ray per lane).  Neighbouring pixels
// have nearly parallel rays, so a wave's 64 gathers per step fall into a
// few cache lines of the map.  A workgroup of WAVES waves covers
// WAVES*tiles_per_wave tiles of one perspective; a perspective with more
// tiles is split over several workgroups whose partial sums are combined in
// fixed point (order independent), the last one writing g_P = sum / N_E
// (Sec. III, IG calculation: the per-perspective mean of the ray gains).
#include <tuple>
#include <type_traits>

#include "ray.hpp"
#include "reduce.hpp"

namespace nbt {

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs, so the
// workgroups of one perspective would land on different L2s.  With a chunk
// C > 0 each XCD instead receives runs of C consecutive logical workgroups
// (runs interleaved across XCDs in launch order, so all XCDs still progress
// through the perspectives together); the incomplete last round keeps the
// identity order.  The mapping is a bijection on [0, nb).
__device__ __forceinline__ uint32_t xcd_logical(uint32_t bid, uint32_t nb, uint32_t chunk) {
    constexpr uint32_t kXcd = 8;
    const uint32_t round = kXcd * chunk;
    const uint32_t full = (nb / round) * round;
    if (bid >= full) return bid;
    const uint32_t xcd = bid % kXcd, slot = bid / kXcd;
    return ((slot / chunk) * kXcd + xcd) * chunk + slot % chunk;
}

// The rays of workgroup-slice g of perspective vp: WAVES waves walk their
// tiles, then the block's sum is written (groups == 1) or combined with the
// other slices of the perspective (last slice writes).  Called uniformly by
// the whole block.  TRACE (parity mode) also writes every ray's record to
// trace[vp * N_E + k], built by the walk below from the offsets it gathers;
// the walk and the IG arithmetic are those of the timed instance.
template <int WAVES, int DEPTH, bool COUNT, bool TRACE>
__device__ __forceinline__ void vp_group(const DevMap& m, const CamParams& c,
                                         const float* __restrict__ pp, uint32_t vp, uint32_t g,
                                         uint32_t groups, uint32_t tiles_x, uint32_t tiles,
                                         int tw_log2, int tpw, float* __restrict__ ig_out,
                                         unsigned long long* __restrict__ steps_out,
                                         VpAccum* __restrict__ ws, nbt_ig_ray_digest* __restrict__ trace) {
    float pose[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) pose[k] = pp[k];

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int tw = 1 << tw_log2;
    const int th = 64 >> tw_log2;
    int lx, ly;
    tile_pixel(lane, tw_log2, lx, ly);
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);

    double acc = 0.0;
    uint32_t steps = 0;
    bool invalid = false;
    for (int r = 0; r < tpw; ++r) {
        const uint32_t tile = (g * WAVES + (uint32_t)wave) * (uint32_t)tpw + (uint32_t)r;
        if (tile >= tiles) break;
        const int i = (int)(tile % tiles_x) * tw + lx;
        const int j = (int)(tile / tiles_x) * th + ly;
        if (i < c.W && j < c.H) {
            RayState ray;
            const int st = setup_ray(m, c, pose, i, j, ray);
            [[maybe_unused]] WalkTrace rec;
            if (st == kRayOk) {
                if constexpr (DEPTH == 1) {
                    if constexpr (TRACE) {
                        // the depth-1 walk addresses each voxel from its coordinates
                        rec.reason = walk_ray<true>(m, rs, ray, acc, steps, [&](int x, int y, int z, uint32_t word) {
                            rec.last = (z * m.ny + y) * m.nx + x;
                            rec.hash = fnv1a_u32(rec.hash, (uint32_t)rec.last);
                            rec.gain += (double)__uint_as_float(word & ~kOccBit);
                            ++rec.steps;
                        });
                    } else {
                        walk_ray<false>(m, rs, ray, acc, steps, [](int, int, int, uint32_t) {});
                    }
                } else {
                    auto walk = [&](auto tl) {
                        constexpr int TLv = decltype(tl)::value;
                        if constexpr (TRACE)
                            walk_ray_pipelined<DEPTH, COUNT, TLv, WalkTrace>(m, rs, ray, acc, steps, &rec);
                        else
                            walk_ray_pipelined<DEPTH, COUNT, TLv>(m, rs, ray, acc, steps);
                    };
                    switch (m.tl) {          // the map's order; uniform per workgroup
                    case 1: walk(std::integral_constant<int, 1>{}); break;
                    case 2: walk(std::integral_constant<int, 2>{}); break;
                    case 3: walk(std::integral_constant<int, 3>{}); break;
                    default: walk(std::integral_constant<int, 0>{});
                    }
                }
            } else if (st == kRayInvalid) {
                invalid = true;
            }
            if constexpr (TRACE)
                write_trace(trace + (size_t)vp * ((size_t)c.W * c.H) + (size_t)j * c.W + i, st, rec);
        }
    }

    acc = wave_sum(acc);
    steps = wave_sum_u32(steps);
    const bool wave_invalid = __ballot(invalid) != 0ull;

    __shared__ double s_acc[WAVES];
    __shared__ unsigned long long s_steps[WAVES];
    __shared__ int s_inv[WAVES];
    if (lane == 0) {
        s_acc[wave] = acc;
        s_steps[wave] = steps;
        s_inv[wave] = wave_invalid ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;

    double tot = 0.0;
    unsigned long long st = 0;
    int inv = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        tot += s_acc[w];
        st += s_steps[w];
        inv |= s_inv[w];
    }
    const double rays = (double)c.W * (double)c.H;
    if (groups == 1) {
        ig_out[vp] = inv ? __builtin_nanf("") : (float)(tot / rays);
        if (steps_out) steps_out[vp] = st;
        return;
    }
    // The slot's fields are only ever touched by device-scope atomic
    // read-modify-writes, which every XCD performs at one point per address
    // (the counts come out exact across XCDs).  Each returned old value is
    // that address's value at the moment this RMW took its place there, so
    // once the three returns are in, this workgroup's sums are part of every
    // later RMW's view.  The count's increment is made to depend on those
    // returns (the empty asm consumes them and hands back the 1), which holds
    // the count's RMW until they have arrived; the last workgroup's count has
    // then come after every other workgroup's sums, and it reads them with
    // RMWs too.  No fence: a release fence at device scope writes back the
    // XCD's L2 in every workgroup, and the last one's acquire fence
    // invalidates it (the map's gathers of the other workgroups there then
    // miss); they cost 8-15 % of a call of 64-256 perspectives of 64x48 rays.
    VpAccum* a = ws + vp;
    const unsigned long long o_sum = atomicAdd(&a->sum_fx, __double2ull_rn(tot * kFixScale));
    const unsigned long long o_steps = atomicAdd(&a->steps, st);
    const unsigned int o_inv = inv ? atomicOr(&a->invalid, 1u) : 0u;
    unsigned int one = 1u;
    asm volatile("" : "+v"(one) : "v"(o_sum), "v"(o_steps), "v"(o_inv));
    const unsigned int done = atomicAdd(&a->count, one);
    if (done == groups - 1) {
        const unsigned long long s = atomicExch(&a->sum_fx, 0ull);
        const unsigned long long stp = atomicExch(&a->steps, 0ull);
        const unsigned int iv = atomicExch(&a->invalid, 0u);
        atomicExch(&a->count, 0u);
        ig_out[vp] = iv ? __builtin_nanf("") : (float)(((double)s / kFixScale) / rays);
        if (steps_out) steps_out[vp] = stp;
    }
}

template <int WAVES, int DEPTH, bool COUNT, bool TRACE>
__global__ __launch_bounds__(WAVES * 64) void ig_viewpoints_kernel(
    DevMap m, CamParams c, const float* __restrict__ poses, uint32_t groups, uint32_t tiles_x,
    uint32_t tiles, int tw_log2, int tpw, int remap, float* __restrict__ ig_out,
    unsigned long long* __restrict__ steps_out, VpAccum* __restrict__ ws,
    nbt_ig_ray_digest* __restrict__ trace) {
    const uint32_t bid = remap > 0 ? xcd_logical(blockIdx.x, gridDim.x, (uint32_t)remap) : blockIdx.x;
    const uint32_t vp = bid / groups;
    const uint32_t g = bid - vp * groups;
    vp_group<WAVES, DEPTH, COUNT, TRACE>(m, c, poses + 12 * (size_t)vp, vp, g, groups, tiles_x, tiles,
                                         tw_log2, tpw, ig_out, steps_out, ws, trace);
}

// Persistent batched launch: many maps, a CSR of perspectives per map
// (offsets[k]..offsets[k+1]).  Work items are (perspective, slice) pairs in
// map-major order; each workgroup pops items from an atomic counter until
// the queue is empty, so uneven maps and perspective counts balance across
// the chip and co-resident workgroups share one map in L2.
template <int WAVES, int DEPTH, bool COUNT>
__global__ __launch_bounds__(WAVES * 64) void ig_batch_kernel(
    const DevMap* __restrict__ maps, uint32_t n_maps, const uint32_t* __restrict__ offsets,
    uint32_t capacity, CamParams c, const float* __restrict__ poses, uint32_t groups,
    uint32_t tiles_x, uint32_t tiles, int tw_log2, int tpw, unsigned int* __restrict__ queue,
    float* __restrict__ ig_out, unsigned long long* __restrict__ steps_out,
    VpAccum* __restrict__ ws) {
    __shared__ uint32_t s_item, s_map;
    uint32_t total = offsets[n_maps];
    total = total < capacity ? total : capacity;
    const uint64_t items = (uint64_t)total * groups;
    for (;;) {
        __syncthreads();                    // previous item's reductions are done
        if (threadIdx.x == 0) {
            const uint32_t it = atomicAdd(queue, 1u);
            uint32_t mi = 0;
            if (it < items) {
                const uint32_t vp = it / groups;
                uint32_t lo = 0, hi = n_maps;          // largest k with offsets[k] <= vp
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) / 2;
                    if (offsets[mid] <= vp) lo = mid; else hi = mid;
                }
                mi = lo;
            }
            s_item = it;
            s_map = mi;
        }
        __syncthreads();
        const uint32_t it = s_item;
        if (it >= items) return;
        const uint32_t vp = it / groups;
        const uint32_t g = it - vp * groups;
        const DevMap m = maps[s_map];
        vp_group<WAVES, DEPTH, COUNT, false>(m, c, poses + 12 * (size_t)vp, vp, g, groups, tiles_x, tiles,
                                             tw_log2, tpw, ig_out, steps_out, ws, nullptr);
    }
}

__global__ void batch_reset_kernel(unsigned int* queue) { *queue = 0u; }

__global__ __launch_bounds__(256) void clear_slots_kernel(VpAccum* __restrict__ ws, uint32_t n) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) ws[i] = VpAccum{0ull, 0ull, 0u, 0u};
}

hipError_t launch_clear_slots(VpAccum* ws, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_slots_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ws, n);
    return hipGetLastError();
}

// Parity mode: one thread per ray, full record per ray.
__global__ __launch_bounds__(256) void trace_rays_kernel(DevMap m, CamParams c,
                                                         const float* __restrict__ poses, uint32_t n,
                                                         nbt_ig_ray_digest* __restrict__ out) {
    const uint64_t rays = (uint64_t)c.W * (uint64_t)c.H;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= rays * n) return;
    const uint32_t vp = (uint32_t)(gid / rays);
    const uint32_t k = (uint32_t)(gid - (uint64_t)vp * rays);
    float pose[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) pose[q] = poses[12 * (size_t)vp + q];
    const int i = (int)(k % (uint32_t)c.W), j = (int)(k / (uint32_t)c.W);

    nbt_ig_ray_digest d;
    d.hash = kFnvBasis;
    d.gain = 0.0;
    d.steps = 0;
    d.stop_lin = -1;
    d.reason = NBT_IG_RAY_MISS;
    d.reserved = 0;
    RayState ray;
    const int st = setup_ray(m, c, pose, i, j, ray);
    if (st == kRayInvalid) {
        d.reason = NBT_IG_RAY_INVALID;
        d.gain = __builtin_nan("");
    } else if (st == kRayOk) {
        unsigned long long h = kFnvBasis;
        int32_t last = -1;
        double acc = 0.0;
        uint32_t steps = 0;
        const int reason = walk_ray<true>(m, map_rsrc(m), ray, acc, steps,
                                          [&](int x, int y, int z, uint32_t) {
                                              last = (z * m.ny + y) * m.nx + x;
                                              h = fnv1a_u32(h, (uint32_t)last);
                                          });
        d.hash = h;
        d.gain = acc;
        d.steps = steps;
        d.stop_lin = last;
        d.reason = (uint32_t)reason;
    }
    out[gid] = d;
}

__global__ __launch_bounds__(256) void trace_paths_kernel(DevMap m, CamParams c,
                                                          const float* __restrict__ poses, uint32_t n,
                                                          const uint32_t* __restrict__ sel,
                                                          uint32_t count, uint32_t max_len,
                                                          int32_t* __restrict__ lin_out,
                                                          uint32_t* __restrict__ len_out) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const uint32_t vp = sel[2 * r], k = sel[2 * r + 1];
    const uint32_t rays = (uint32_t)c.W * (uint32_t)c.H;
    if (vp >= n || k >= rays) {
        len_out[r] = 0;
        return;
    }
    float pose[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) pose[q] = poses[12 * (size_t)vp + q];
    RayState ray;
    uint32_t steps = 0;
    if (setup_ray(m, c, pose, (int)(k % (uint32_t)c.W), (int)(k / (uint32_t)c.W), ray) == kRayOk) {
        double acc = 0.0;
        int32_t* dst = lin_out + (size_t)r * max_len;
        uint32_t w = 0;
        walk_ray<true>(m, map_rsrc(m), ray, acc, steps, [&](int x, int y, int z, uint32_t) {
            if (w < max_len) dst[w] = (z * m.ny + y) * m.nx + x;
            ++w;
        });
    }
    len_out[r] = steps;
}

hipError_t launch_eval_viewpoints(const DevMap& m, const CamParams& c, const float* poses,
                                  uint32_t n, float* ig_out, unsigned long long* steps_out,
                                  VpAccum* ws, const VpLaunch& L0, hipStream_t s,
                                  nbt_ig_ray_digest* trace) {
    const VpLaunch L = resolve_launch(c, L0);
    const int tw = 1 << L.tile_w_log2, th = 64 >> L.tile_w_log2;
    const uint32_t tiles_x = (uint32_t)((c.W + tw - 1) / tw);
    const uint32_t tiles = tiles_x * (uint32_t)((c.H + th - 1) / th);
    const uint32_t groups = vp_groups(c, L);
    const dim3 grid((unsigned)((uint64_t)n * groups));
    const auto args = std::make_tuple(m, c, poses, groups, tiles_x, tiles, L.tile_w_log2,
                                      L.tiles_per_wave, L.xcd_remap, ig_out, steps_out, ws, trace);
    auto go = [&](auto kernel, int waves) {
        std::apply([&](auto... a) { hipLaunchKernelGGL(kernel, grid, dim3(waves * 64), 0, s, a...); },
                   args);
    };
    // Without steps_out the walk skips the per-voxel visit count.
    const bool count = steps_out != nullptr;
#define NBT_VP_GO(W, D)                                                                            \
    (trace ? (count ? go(ig_viewpoints_kernel<W, D, true, true>, W)                                \
                    : go(ig_viewpoints_kernel<W, D, false, true>, W))                              \
           : (count ? go(ig_viewpoints_kernel<W, D, true, false>, W)                               \
                    : go(ig_viewpoints_kernel<W, D, false, false>, W)))
#define NBT_VP_DEPTHS(W)                                  \
    case W:                                               \
        switch (L.depth) {                                \
            case 1: NBT_VP_GO(W, 1); break;               \
            case 2: NBT_VP_GO(W, 2); break;               \
            case 4: NBT_VP_GO(W, 4); break;               \
            case 8: NBT_VP_GO(W, 8); break;               \
            default: return hipErrorInvalidValue;         \
        }                                                 \
        break;
    switch (L.waves) {
        NBT_VP_DEPTHS(1)
        NBT_VP_DEPTHS(2)
        NBT_VP_DEPTHS(4)
        NBT_VP_DEPTHS(8)
        default:
            return hipErrorInvalidValue;
    }
#undef NBT_VP_GO
#undef NBT_VP_DEPTHS
    return hipGetLastError();
}

const void* batch_kernel_ptr(int waves, int depth, bool count) {
#define NBT_BK(W, D)                                                                      \
    if (waves == W && depth == D)                                                         \
        return count ? (const void*)ig_batch_kernel<W, D, true> : (const void*)ig_batch_kernel<W, D, false>;
    NBT_BK(1, 1) NBT_BK(1, 2) NBT_BK(1, 4) NBT_BK(1, 8)
    NBT_BK(2, 1) NBT_BK(2, 2) NBT_BK(2, 4) NBT_BK(2, 8)
    NBT_BK(4, 1) NBT_BK(4, 2) NBT_BK(4, 4) NBT_BK(4, 8)
    NBT_BK(8, 1) NBT_BK(8, 2) NBT_BK(8, 4) NBT_BK(8, 8)
#undef NBT_BK
    return nullptr;
}

const void* batch_reset_ptr() { return (const void*)batch_reset_kernel; }

hipError_t launch_trace_rays(const DevMap& m, const CamParams& c, const float* poses, uint32_t n,
                             nbt_ig_ray_digest* out, hipStream_t s) {
    const uint64_t total = (uint64_t)c.W * c.H * n;
    const uint64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(trace_rays_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, c, poses, n, out);
    return hipGetLastError();
}

hipError_t launch_trace_paths(const DevMap& m, const CamParams& c, const float* poses, uint32_t n,
                              const uint32_t* rays, uint32_t count, uint32_t max_len,
                              int32_t* lin_out, uint32_t* len_out, hipStream_t s) {
    const uint32_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(trace_paths_kernel, dim3(blocks), dim3(256), 0, s, m, c, poses, n, rays,
                       count, max_len, lin_out, len_out);
    return hipGetLastError();
}

}  // namespace nbt
