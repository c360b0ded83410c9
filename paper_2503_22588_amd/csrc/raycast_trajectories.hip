// raycast_trajectories.hip -- union information gain of camera trajectories.
//
// A trajectory of L poses sees the union U of the voxels visited by all rays
// of all its poses; each voxel counts once however many rays or poses meet it
// (a voxel seen again along the path brings no new information).  One
// workgroup owns one trajectory and keeps U as a bitset over the voxel box
// that contains every frustum of the trajectory:
//   1. a pre-pass computes the box per trajectory (apex + 4 far-plane corners
//      per pose, one voxel of margin, clipped to the map) and routes boxes
//      that fit the LDS budget to the LDS kernel, the rest to global memory;
//   2. the union kernel walks all L x N_E rays (one ray per lane, 8x8 tiles
//      per wave, pipelined gathers) and sets one bit per visited voxel with
//      an atomic OR (idempotent, so the set does not depend on thread order;
//      in LDS only bits found unset take the atomic);
//   3. the epilogue scans the bitset in a fixed order: |U|, per-state counts
//      (exact integers) and the summed Eq. 2 gains of U (binary64).
#include <tuple>

#include "internal.hpp"
#include "ray.hpp"
#include "reduce.hpp"

namespace nbt {

// dda_advance plus a second index (a bitset position) that moves with the
// map offset: by dbx/dby/dbz per step on x/y/z.  Past the segment end it
// drifts, but every slot from there on reads the sentinel and is never
// marked, so it needs no gating.
template <int TL>
__device__ __forceinline__ void dda_advance_idx(float& tx, float& ty, float& tz, uint32_t& off,
                                                int& idx, bool& alive, float t1, int dxo, int dyo, int dzo,
                                                int bxo, int byo, uint32_t flip, int dbx, int dby,
                                                int dbz, float dtx, float dty, float dtz) {
    const float x = tx, y = ty, z = tz;
    const float tm = fminf(fminf(x, y), z);
    const bool go = alive && !(tm > t1);
    const bool ex = x == tm, ey = y == tm;
    const bool bx = go && ex;
    const bool by = go && !ex && ey;
    const bool bz = go && !ex && !ey;
    int d;
    if constexpr (TL != 0) {
        const uint32_t msk = bx ? tile_mask_x<TL>() : tile_mask_y<TL>();
        const int big = bx ? bxo : byo;
        const int small = bx ? dxo : dyo;
        const int dxy = ((off ^ flip) & msk) == 0u ? big : small;
        d = bz ? dzo : dxy;
    } else {
        d = bx ? dxo : (by ? dyo : dzo);
    }
    off = go ? off + (uint32_t)d : 0u;
    idx += bx ? dbx : (by ? dby : dbz);
    // the stepping axis gains its delta, the others add +0 (t >= 0, so exact):
    // three selects and three adds instead of five selects and one add
    tx = x + (bx ? dtx : 0.0f);
    ty = y + (by ? dty : 0.0f);
    tz = z + (bz ? dtz : 0.0f);
    alive = go;
}

// Pipelined walk that also sets, in `bits`, the bit of every visited voxel of
// the box [lo, lo + (ax, ay, *)): ((z-lz)*ay + (y-ly))*ax + (x-lx).  Indices
// at or beyond nbits (a voxel outside the box, impossible when the box
// contains the ray's frustum) are not counted.
//
// CHECK (bitsets in LDS): along a trajectory almost every visit finds its bit
// already set, so a slot reads the word and only an unset bit costs an atomic
// OR; the read of slot u is checked one slot later, which keeps its latency
// off the walk.  Setting a bit twice is harmless, and a stale read can only
// show fewer bits than are set, so the set of marked voxels is exactly the set
// visited.  The bitset is preceded by one all-ones word (bits[-1]): a slot
// that marks nothing reads it and never calls for the atomic.  An index at or
// beyond nbits is clamped to bit nbits (the bitset has nbits / 32 + 1 words,
// so that bit exists), which the epilogue ignores.  One select per slot, where
// a compare, two selects and a mask operation would otherwise decide the mark.
//
// CHECK = false (bitsets in global memory, where a read could be served by a
// stale L1 line): every visit sets its bit with an atomic OR.
//
// Returns the number of voxels visited when COUNT is set (0 otherwise:
// without a per-lane count the loop is guarded by a group budget, as in
// walk_ray_pipelined).
template <int P, bool CHECK, int TL, bool COUNT>
__device__ __forceinline__ uint32_t walk_ray_mark(const DevMap& m, __amdgpu_buffer_rsrc_t rs,
                                                  const RayState& r, int lx, int ly, int lz, int ax,
                                                  int ay, uint32_t nbits, uint32_t* bits) {
    const OffsetSteps o = offset_steps<TL>(m, r);
    const int dbx = r.sx, dby = r.sy * ax, dbz = r.sz * ax * ay;
    const float dtx = r.dtx, dty = r.dty, dtz = r.dtz;
    const float t1 = r.t1;
    uint32_t off = voxel_offset(m, r.ix, r.iy, r.iz);
    int bidx = ((r.iz - lz) * ay + (r.iy - ly)) * ax + (r.ix - lx);
    float tx = r.tx, ty = r.ty, tz = r.tz;
    const uint32_t guard = (uint32_t)(m.nx + m.ny + m.nz + 3);
    uint32_t budget = guard / P + 2;
    bool alive = true;

    uint32_t w[P];
    int bi[P];
    w[0] = load_word(rs, off);
    bi[0] = bidx;
#pragma unroll
    for (int u = 1; u < P; ++u) {
        dda_advance_idx<TL>(tx, ty, tz, off, bidx, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                               dbx, dby, dbz, dtx, dty, dtz);
        w[u] = load_word(rs, off);
        bi[u] = bidx;
    }
    uint32_t n = 0;
    bool run = true;
    int pend_word = -1;                                       // the previous slot's mark
    uint32_t pend_mask = 0, pend_seen = 0;
    // Same slot structure as walk_ray_pipelined.
    while (run) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const uint32_t x = w[u];
            const bool take = run && x != kSentinel;
            if constexpr (CHECK) {
                if (pend_mask & ~pend_seen) atomicOr(&bits[pend_word], pend_mask);
                const uint32_t b = min((uint32_t)bi[u], nbits);
                pend_word = take ? (int)(b >> 5) : -1;
                pend_mask = 1u << (b & 31u);
                pend_seen = bits[pend_word];
                // keep this slot's generator step after the read, so that the
                // read has the step's latency to complete before it is checked
                __builtin_amdgcn_sched_barrier(0);
            } else if (take && (uint32_t)bi[u] < nbits) {
                atomicOr(&bits[(uint32_t)bi[u] >> 5], 1u << ((uint32_t)bi[u] & 31u));
            }
            if constexpr (COUNT) n += take ? 1u : 0u;
            run = run && (int)x >= 0;
            dda_advance_idx<TL>(tx, ty, tz, off, bidx, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                               dbx, dby, dbz, dtx, dty, dtz);
            w[u] = load_word(rs, off);
            bi[u] = bidx;
        }
        // the border bounds the visits below nx + ny + nz; the guards only back that up
        if constexpr (COUNT) run = run && n < guard;
        else run = run && --budget != 0u;
    }
    if constexpr (CHECK)
        if (pend_mask & ~pend_seen) atomicOr(&bits[pend_word], pend_mask);
    return n;
}

__global__ __launch_bounds__(256) void traj_box_kernel(DevMap m, CamParams c,
                                                       const float* __restrict__ poses, uint32_t T,
                                                       uint32_t L, uint32_t budget_bits,
                                                       TrajBox* __restrict__ boxes,
                                                       TrajMeta* __restrict__ meta,
                                                       uint32_t* __restrict__ over_list) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const float org[3] = {m.ox, m.oy, m.oz};
    const int n[3] = {m.nx, m.ny, m.nz};
    const float u_lo = c.W > 1 ? -c.dh : 0.0f, u_hi = c.W > 1 ? c.dh : 0.0f;
    const float v_lo = c.H > 1 ? -c.dv : 0.0f, v_hi = c.H > 1 ? c.dv : 0.0f;
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    bool unbounded = false;
    for (uint32_t l = 0; l < L; ++l) {
        const float* p = poses + 12 * ((size_t)t * L + l);
        for (int q = 0; q < 5; ++q) {
            const float u = q == 0 ? 0.0f : ((q & 1) ? u_lo : u_hi);
            const float v = q == 0 ? 0.0f : ((q & 2) ? v_lo : v_hi);
            const float d = q == 0 ? 0.0f : c.range;
            for (int a = 0; a < 3; ++a) {
                float w = p[3 * a + 0] * u;
                w = w + p[3 * a + 1] * v;
                w = w + p[3 * a + 2] * d;
                const float e = (q == 0) ? p[9 + a] : p[9 + a] + w;
                const float vx = (e - org[a]) * m.inv_s;
                if (!__builtin_isfinite(vx)) unbounded = true;
                lo[a] = vx < lo[a] ? vx : lo[a];
                hi[a] = vx > hi[a] ? vx : hi[a];
            }
        }
    }
    int ilo[3], ihi[3];
    for (int a = 0; a < 3; ++a) {
        if (unbounded) {
            ilo[a] = 0;
            ihi[a] = n[a] - 1;
        } else {
            const float fl = floorf(lo[a]) - 1.0f, fh = floorf(hi[a]) + 1.0f;
            const float cl = fl < 0.0f ? 0.0f : (fl > (float)(n[a] - 1) ? (float)(n[a] - 1) : fl);
            const float ch = fh < 0.0f ? 0.0f : (fh > (float)(n[a] - 1) ? (float)(n[a] - 1) : fh);
            ilo[a] = (int)cl;
            ihi[a] = (int)ch;
        }
    }
    TrajBox b;
    b.lx = ilo[0]; b.ly = ilo[1]; b.lz = ilo[2];
    b.ax = ihi[0] - ilo[0] + 1; b.ay = ihi[1] - ilo[1] + 1; b.az = ihi[2] - ilo[2] + 1;
    b.nbits = (L == 0) ? 0u : (uint32_t)b.ax * (uint32_t)b.ay * (uint32_t)b.az;
    b.global = 0;
    b.goff = 0;
    if (b.nbits <= budget_bits) {
        atomicMax(&meta->max_bits, b.nbits);
    } else {
        b.global = 1;
        const unsigned long long words = ((unsigned long long)b.nbits + 31) / 32;
        b.goff = atomicAdd(&meta->global_words, (words + 63) / 64 * 64);
        over_list[atomicAdd(&meta->n_global, 1u)] = t;
    }
    boxes[t] = b;
}

// Eight waves per SIMD: the kernel fits 64 VGPRs, and left to itself the
// compiler took 106 SGPRs, which allow only seven; with the hint it keeps 78
// (the few spills are outside the walk) and four 8-wave workgroups fit a CU.
template <bool GLOBAL, int WAVES, bool COUNT>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(8, 8))) void traj_union_kernel(
    DevMap m, CamParams c, const float* __restrict__ poses, uint32_t L,
    const TrajBox* __restrict__ boxes, const uint32_t* __restrict__ over_list,
    uint32_t* __restrict__ gbits, float* __restrict__ ig_union, uint32_t* __restrict__ counts,
    unsigned long long* __restrict__ visits) {
    extern __shared__ uint32_t lds_bits[];
    const uint32_t t = GLOBAL ? over_list[blockIdx.x] : blockIdx.x;
    const TrajBox b = boxes[t];
    if (!GLOBAL && b.global) return;
    // in LDS the bitset follows the walk's all-ones word and holds bit nbits
    uint32_t* bits = GLOBAL ? gbits + b.goff : lds_bits + 1;
    const uint32_t nwords = GLOBAL ? (b.nbits + 31) / 32 : b.nbits / 32 + 1;
    const uint32_t tid = threadIdx.x;
    for (uint32_t w = tid; w < nwords; w += blockDim.x) bits[w] = 0u;
    if (!GLOBAL && tid == 0) lds_bits[0] = ~0u;
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    int lx, ly;
    tile_pixel(lane, 3, lx, ly);
    const uint32_t tiles_x = (uint32_t)(c.W + 7) / 8;
    const uint32_t tiles_pose = tiles_x * (uint32_t)((c.H + 7) / 8);
    const uint32_t total = tiles_pose * L;
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);
    uint32_t steps = 0;
    bool invalid = false;
    for (uint32_t tile = (uint32_t)wave; tile < total; tile += WAVES) {
        const uint32_t l = tile / tiles_pose;
        const uint32_t tt = tile - l * tiles_pose;
        const float* pp = poses + 12 * ((size_t)t * L + l);
        float pose[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) pose[k] = pp[k];
        const int i = (int)(tt % tiles_x) * 8 + lx;
        const int j = (int)(tt / tiles_x) * 8 + ly;
        if (i < c.W && j < c.H) {
            RayState ray;
            const int st = setup_ray(m, c, pose, i, j, ray);
            if (st == kRayOk) {
                switch (m.tl) {                  // the map's order; uniform per workgroup
                case 1:
                    steps += walk_ray_mark<4, !GLOBAL, 1, COUNT>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay, b.nbits,
                                                                 bits);
                    break;
                case 2:
                    steps += walk_ray_mark<4, !GLOBAL, 2, COUNT>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay, b.nbits,
                                                                 bits);
                    break;
                case 3:
                    steps += walk_ray_mark<4, !GLOBAL, 3, COUNT>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay, b.nbits,
                                                                 bits);
                    break;
                default:
                    steps += walk_ray_mark<4, !GLOBAL, 0, COUNT>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay, b.nbits,
                                                                 bits);
                }
            } else if (st == kRayInvalid) {
                invalid = true;
            }
        }
    }
    __syncthreads();

    // Epilogue: classify the voxels of U from their encoded words.
    uint32_t c_occ = 0, c_free = 0, c_unk = 0;
    double gain = 0.0;
    const int axy = b.ax * b.ay;
    for (uint32_t w = tid; w < nwords; w += blockDim.x) {
        uint32_t word = GLOBAL ? __hip_atomic_load(&bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : bits[w];
        // bits at or beyond nbits (the walk's clamp target) are not voxels of the box
        if (w == b.nbits >> 5) word &= (1u << (b.nbits & 31u)) - 1u;
        while (word) {
            const int bit = __ffs(word) - 1;
            word &= word - 1u;
            const int idx = (int)(w * 32u) + bit;
            const int z = idx / axy;
            const int rem = idx - z * axy;
            const int y = rem / b.ax;
            const int x = rem - y * b.ax;
            const uint32_t e = load_word(rs, voxel_offset(m, b.lx + x, b.ly + y, b.lz + z));
            gain += (double)__uint_as_float(e & ~kOccBit);
            if (e & kOccBit) ++c_occ;
            else if (e == kGainOne) ++c_unk;
            else ++c_free;
        }
    }
    gain = wave_sum(gain);
    c_occ = wave_sum_u32(c_occ);
    c_free = wave_sum_u32(c_free);
    c_unk = wave_sum_u32(c_unk);
    const unsigned long long st = wave_sum_u64((unsigned long long)steps);
    const bool wave_invalid = __ballot(invalid) != 0ull;
    __shared__ double s_gain[WAVES];
    __shared__ unsigned long long s_steps[WAVES];
    __shared__ uint32_t s_cnt[WAVES][3];
    __shared__ int s_inv[WAVES];
    if (lane == 0) {
        s_gain[wave] = gain;
        s_steps[wave] = st;
        s_cnt[wave][0] = c_occ;
        s_cnt[wave][1] = c_free;
        s_cnt[wave][2] = c_unk;
        s_inv[wave] = wave_invalid ? 1 : 0;
    }
    __syncthreads();
    if (tid != 0) return;
    double g = 0.0;
    unsigned long long vs = 0;
    uint32_t co = 0, cf = 0, cu = 0;
    int inv = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        g += s_gain[w];
        vs += s_steps[w];
        co += s_cnt[w][0];
        cf += s_cnt[w][1];
        cu += s_cnt[w][2];
        inv |= s_inv[w];
    }
    ig_union[t] = inv ? __builtin_nanf("") : (float)g;
    counts[4 * (size_t)t + 0] = co + cf + cu;
    counts[4 * (size_t)t + 1] = co;
    counts[4 * (size_t)t + 2] = cf;
    counts[4 * (size_t)t + 3] = cu;
    if (visits) visits[t] = vs;
}

size_t traj_static_lds_bytes() {
    // the largest static LDS among the workgroup sizes (the 16-wave kernel)
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void*)traj_union_kernel<false, 16, true>) != hipSuccess) return 4096;
    return a.sharedSizeBytes;
}

hipError_t launch_traj_boxes(const DevMap& m, const CamParams& c, const float* poses, uint32_t T,
                             uint32_t L, uint32_t budget_bits, TrajBox* boxes, TrajMeta* meta,
                             uint32_t* over_list, hipStream_t s) {
    // budget_bits is the LDS a bitset may take.  An LDS bitset of b bits has
    // b / 32 + 1 words after the walk's all-ones word, at most
    // ceil(b / 32) * 4 + 8 bytes (launch_union adds the 8): boxes are routed
    // to LDS only while that fits.
    const uint32_t words = budget_bits / 32;
    const uint32_t fit_bits = words > 2 ? (words - 2) * 32 : 0;
    hipLaunchKernelGGL(traj_box_kernel, dim3((T + 255) / 256), dim3(256), 0, s, m, c, poses, T, L,
                       fit_bits, boxes, meta, over_list);
    return hipGetLastError();
}

template <bool GLOBAL, int WAVES, bool COUNT>
static hipError_t launch_union(const DevMap& m, const CamParams& c, const float* poses, uint32_t L,
                               uint32_t grid, size_t lds_bytes, const TrajBox* boxes,
                               const uint32_t* over_list, uint32_t* gbits, float* ig_union,
                               uint32_t* counts, unsigned long long* visits, hipStream_t s) {
    const void* k = (const void*)traj_union_kernel<GLOBAL, WAVES, COUNT>;
    // lds_bytes covers ceil(max_bits / 32) words; the all-ones word and the
    // word that holds bit max_bits come on top
    const size_t lds = GLOBAL ? 0 : lds_bytes + 8;
    if (!GLOBAL) {
        static std::atomic<size_t> lds_set[64];
        const hipError_t e = allow_dynamic_lds(k, lds, lds_set, 64);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((traj_union_kernel<GLOBAL, WAVES, COUNT>), dim3(grid), dim3(WAVES * 64), lds,
                       s, m, c, poses, L, boxes, over_list, gbits, ig_union, counts, visits);
    return hipGetLastError();
}

hipError_t launch_traj_union(bool global, int waves, const DevMap& m, const CamParams& c,
                             const float* poses, uint32_t L, uint32_t grid, size_t lds_bytes,
                             const TrajBox* boxes, const uint32_t* over_list, uint32_t* gbits,
                             float* ig_union, uint32_t* counts, unsigned long long* visits,
                             hipStream_t s) {
    const bool count = visits != nullptr;    // no visit count when the caller does not ask for it
#define NBT_TU(G, W, C)                                                                              \
    if (global == G && waves == W && count == C)                                                     \
        return launch_union<G, W, C>(m, c, poses, L, grid, lds_bytes, boxes, over_list, gbits, ig_union, \
                                     counts, visits, s);
    NBT_TU(false, 4, true) NBT_TU(false, 8, true) NBT_TU(false, 16, true)
    NBT_TU(true, 4, true) NBT_TU(true, 8, true) NBT_TU(true, 16, true)
    NBT_TU(false, 4, false) NBT_TU(false, 8, false) NBT_TU(false, 16, false)
    NBT_TU(true, 4, false) NBT_TU(true, 8, false) NBT_TU(true, 16, false)
#undef NBT_TU
    return hipErrorInvalidValue;
}

}  // namespace nbt
