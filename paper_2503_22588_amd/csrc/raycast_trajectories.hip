// raycast_trajectories.hip -- union information gain of camera trajectories.
//
// A trajectory of L poses sees the union U of the voxels visited by all rays
// of all its poses; each voxel counts once however many rays or poses meet it
// (a voxel seen again along the path brings no new information).  One
// workgroup owns one trajectory and keeps U as a bitset over the voxel box
// that contains every frustum of the trajectory:
//   1. a pre-pass computes the box per trajectory (apex + 4 far-plane corners
//      per pose, one voxel of margin, clipped to the map);
//   2. the union kernel walks all L x N_E rays (one ray per lane, 8x8 tiles
//      per wave, pipelined gathers) and sets one LDS bit per visited voxel
//      with an atomic OR where a read finds it unset (idempotent, so the set
//      does not depend on thread order); a box larger than the LDS slice is
//      covered in several passes over the rays, one slice of it per pass;
//   3. the epilogue scans the bitset in a fixed order: |U|, per-state counts
//      (exact integers) and the summed Eq. 2 gains of U (binary64).
// Both launches are sized from the call's arguments alone: nothing is read
// back to the host, so a call can be captured in a graph.
#include <tuple>

#include "internal.hpp"
#include "ray.hpp"
#include "reduce.hpp"

namespace nbt {

// Canonical linear index of box position `idx` of the box at (lx, ly, lz)
// with extent (ax, ay, *) (x fastest) and box_bits positions; -1 outside the
// box or the map.  Parity mode only.
__device__ __forceinline__ int32_t box_lin(const DevMap& m, int lx, int ly, int lz, int ax, int ay,
                                           uint32_t box_bits, int idx) {
    if (idx < 0 || (uint32_t)idx >= box_bits) return -1;
    const int x = lx + idx % ax, y = ly + (idx / ax) % ay, z = lz + idx / (ax * ay);
    if (x >= m.nx || y >= m.ny || z >= m.nz) return -1;
    return (z * m.ny + y) * m.nx + x;
}

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

// Pipelined walk that also sets, in the LDS bitset `bits`, the bit of every
// visited voxel whose box position ((z-lz)*ay + (y-ly))*ax + (x-lx), minus
// `base`, lies in [0, nbits): the slice of the box one pass of the union
// kernel marks.  Positions outside the slice (earlier or later passes, or a
// voxel outside the box, impossible when the box contains the ray's frustum)
// are clamped to bit nbits, which the bitset holds (it has nbits / 32 + 1
// words) and the epilogue ignores.
//
// Along a trajectory almost every visit finds its bit already set, so a slot
// reads the word and only an unset bit costs an atomic OR; the read of slot u
// is checked one slot later, which keeps its latency off the walk.  Setting a
// bit twice is harmless, and a stale read can only show fewer bits than are
// set, so the set of marked voxels is exactly the set visited.  The bitset is
// preceded by one all-ones word (bits[-1]): a slot that marks nothing reads it
// and never calls for the atomic.  One select and one min per slot decide the
// mark, where a compare, two selects and a mask operation would otherwise.
//
// Returns the number of voxels visited when COUNT is set (0 otherwise:
// without a per-lane count the loop is guarded by a group budget, as in
// walk_ray_pipelined).  With TR = WalkTrace the record also checks every
// visit's bitset position against the voxel its gather read.
template <int P, int TL, bool COUNT, class TR = NoTrace>
__device__ __forceinline__ uint32_t walk_ray_mark(const DevMap& m, __amdgpu_buffer_rsrc_t rs,
                                                  const RayState& r, int lx, int ly, int lz, int ax,
                                                  int ay, int base, uint32_t nbits, uint32_t* bits,
                                                  TR* tr = nullptr) {
    const OffsetSteps o = offset_steps<TL>(m, r);
    const int dbx = r.sx, dby = r.sy * ax, dbz = r.sz * ax * ay;
    const float dtx = r.dtx, dty = r.dty, dtz = r.dtz;
    const float t1 = r.t1;
    uint32_t off = voxel_offset(m, r.ix, r.iy, r.iz);
    int bidx = ((r.iz - lz) * ay + (r.iy - ly)) * ax + (r.ix - lx) - base;
    float tx = r.tx, ty = r.ty, tz = r.tz;
    const uint32_t guard = (uint32_t)(m.nx + m.ny + m.nz + 3);
    uint32_t budget = guard / P + 2;
    bool alive = true;

    uint32_t w[P];
    int bi[P];
    [[maybe_unused]] uint32_t wo[P];          // parity mode only (see walk_ray_pipelined)
    [[maybe_unused]] bool wl[P];
    w[0] = load_word(rs, off);
    bi[0] = bidx;
    if constexpr (traced<TR>()) {
        wo[0] = off;
        wl[0] = true;
    }
#pragma unroll
    for (int u = 1; u < P; ++u) {
        dda_advance_idx<TL>(tx, ty, tz, off, bidx, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                               dbx, dby, dbz, dtx, dty, dtz);
        w[u] = load_word(rs, off);
        bi[u] = bidx;
        if constexpr (traced<TR>()) {
            wo[u] = off;
            wl[u] = alive;
        }
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
            if (pend_mask & ~pend_seen) atomicOr(&bits[pend_word], pend_mask);
            const uint32_t b = min((uint32_t)bi[u], nbits);
            pend_word = take ? (int)(b >> 5) : -1;
            pend_mask = 1u << (b & 31u);
            pend_seen = bits[pend_word];
            // keep this slot's generator step after the read, so that the
            // read has the step's latency to complete before it is checked
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (COUNT) n += take ? 1u : 0u;
            if constexpr (traced<TR>()) {
                if (run) {
                    tr->consume(m, x, wo[u], wl[u], t1);
                    if (x != kSentinel && box_lin(m, lx, ly, lz, ax, ay, tr->box_bits, bi[u] + base) != tr->last)
                        ++tr->mismatch;
                }
            }
            run = run && (int)x >= 0;
            dda_advance_idx<TL>(tx, ty, tz, off, bidx, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                               dbx, dby, dbz, dtx, dty, dtz);
            w[u] = load_word(rs, off);
            bi[u] = bidx;
            if constexpr (traced<TR>()) {
                wo[u] = off;
                wl[u] = alive;
            }
        }
        // the border bounds the visits below nx + ny + nz; the guards only back that up
        if constexpr (COUNT) run = run && n < guard;
        else run = run && --budget != 0u;
    }
    if (pend_mask & ~pend_seen) atomicOr(&bits[pend_word], pend_mask);
    if constexpr (traced<TR>()) tr->finish();
    return n;
}

__global__ __launch_bounds__(256) void traj_box_kernel(DevMap m, CamParams c,
                                                       const float* __restrict__ poses, uint32_t T,
                                                       uint32_t L, TrajBox* __restrict__ boxes) {
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
    boxes[t] = b;
}

// One workgroup per trajectory.  The bitset of its box is kept in LDS,
// `pass_words` 32-bit words at a time: a box of more bits is covered in
// several passes, each walking all rays again and marking only its slice of
// the box's positions.  The epilogue of every pass hands word w of the whole
// box to thread w mod blockDim, in increasing w, so the counts and the summed
// gains (binary64) are the same bits whatever the number of passes.
//
// Eight waves per SIMD: the kernel fits 64 VGPRs, and left to itself the
// compiler took 106 SGPRs, which allow only seven; with the hint it keeps 78
// (the few spills are outside the walk) and four 8-wave workgroups fit a CU.
template <int WAVES, bool COUNT, bool TRACE>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(8, 8))) void traj_union_kernel(
    DevMap m, CamParams c, const float* __restrict__ poses, uint32_t L,
    const TrajBox* __restrict__ boxes, uint32_t pass_words, float* __restrict__ ig_union,
    uint32_t* __restrict__ counts, unsigned long long* __restrict__ visits,
    nbt_ig_ray_digest* __restrict__ trace) {
    extern __shared__ uint32_t lds_bits[];
    const uint32_t t = blockIdx.x;
    const TrajBox b = boxes[t];
    // the bitset follows the walk's all-ones word and holds the clamp bit
    uint32_t* bits = lds_bits + 1;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthreads = WAVES * 64;
    const uint32_t pass_bits = pass_words * 32u;
    const uint32_t passes = b.nbits == 0 ? 1u : (b.nbits - 1u) / pass_bits + 1u;
    if (tid == 0) lds_bits[0] = ~0u;

    const int wave = tid >> 6, lane = tid & 63;
    int lx, ly;
    tile_pixel(lane, 3, lx, ly);
    const uint32_t tiles_x = (uint32_t)(c.W + 7) / 8;
    const uint32_t tiles_pose = tiles_x * (uint32_t)((c.H + 7) / 8);
    const uint32_t total = tiles_pose * L;
    const uint64_t rays = (uint64_t)c.W * (uint64_t)c.H;
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);
    uint32_t steps = 0;
    bool invalid = false;
    uint32_t c_occ = 0, c_free = 0, c_unk = 0;
    double gain = 0.0;
    const int axy = b.ax * b.ay;

    for (uint32_t pass = 0; pass < passes; ++pass) {
        const uint32_t base = pass * pass_bits;
        const uint32_t nb = min(pass_bits, b.nbits - base);     // bits of this slice
        for (uint32_t w = tid; w <= nb / 32u; w += nthreads) bits[w] = 0u;
        __syncthreads();

        for (uint32_t tile = (uint32_t)wave; tile < total; tile += WAVES) {
            // poses fastest: a workgroup's waves walk the same pixel tile of
            // consecutive poses together, whose rays meet mostly the same voxels
            const uint32_t tt = tile / L;
            const uint32_t l = tile - tt * L;
            const float* pp = poses + 12 * ((size_t)t * L + l);
            float pose[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) pose[k] = pp[k];
            const int i = (int)(tt % tiles_x) * 8 + lx;
            const int j = (int)(tt / tiles_x) * 8 + ly;
            if (i < c.W && j < c.H) {
                RayState ray;
                const int st = setup_ray(m, c, pose, i, j, ray);
                WalkTrace rec;
                rec.box_bits = b.nbits;
                if (st == kRayOk) {
                    uint32_t n;
                    auto walk = [&](auto tl) {
                        constexpr int TLv = decltype(tl)::value;
                        if constexpr (TRACE)
                            return walk_ray_mark<4, TLv, COUNT, WalkTrace>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay,
                                                                          (int)base, nb, bits, &rec);
                        else
                            return walk_ray_mark<4, TLv, COUNT>(m, rs, ray, b.lx, b.ly, b.lz, b.ax, b.ay,
                                                               (int)base, nb, bits);
                    };
                    switch (m.tl) {                  // the map's order; uniform per workgroup
                    case 1: n = walk(std::integral_constant<int, 1>{}); break;
                    case 2: n = walk(std::integral_constant<int, 2>{}); break;
                    case 3: n = walk(std::integral_constant<int, 3>{}); break;
                    default: n = walk(std::integral_constant<int, 0>{});
                    }
                    if (pass == 0) steps += n;
                } else if (st == kRayInvalid) {
                    invalid = true;
                }
                if constexpr (TRACE) {
                    if (pass == 0)
                        write_trace(trace + ((size_t)t * L + l) * rays + (size_t)j * c.W + i, st, rec);
                }
            }
        }
        __syncthreads();

        // Epilogue of the slice: classify the voxels of U from their encoded words.
        const uint32_t base_w = base / 32u;                      // pass_bits is a multiple of 32
        const uint32_t nw = (nb + 31u) / 32u;
        uint32_t w = (tid + nthreads - base_w % nthreads) % nthreads;   // first word of this thread
        for (; w < nw; w += nthreads) {
            uint32_t word = bits[w];
            // bits at or beyond nb (the walk's clamp target) are not voxels of the slice
            if (w == nb >> 5) word &= (1u << (nb & 31u)) - 1u;
            while (word) {
                const int bit = __ffs(word) - 1;
                word &= word - 1u;
                const int idx = (int)(base + w * 32u) + bit;
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
        __syncthreads();       // the next pass clears the bitset
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
    if (hipFuncGetAttributes(&a, (const void*)traj_union_kernel<16, true, true>) != hipSuccess) return 4096;
    return a.sharedSizeBytes;
}

const void* traj_union_kernel_ptr(int waves) {
    switch (waves) {
    case 4: return (const void*)traj_union_kernel<4, false, false>;
    case 8: return (const void*)traj_union_kernel<8, false, false>;
    case 16: return (const void*)traj_union_kernel<16, false, false>;
    default: return nullptr;
    }
}

hipError_t launch_traj_boxes(const DevMap& m, const CamParams& c, const float* poses, uint32_t T,
                             uint32_t L, TrajBox* boxes, hipStream_t s) {
    hipLaunchKernelGGL(traj_box_kernel, dim3((T + 255) / 256), dim3(256), 0, s, m, c, poses, T, L, boxes);
    return hipGetLastError();
}

template <int WAVES, bool COUNT, bool TRACE>
static hipError_t launch_union(const DevMap& m, const CamParams& c, const float* poses, uint32_t L,
                               uint32_t T, uint32_t pass_words, const TrajBox* boxes, float* ig_union,
                               uint32_t* counts, unsigned long long* visits, nbt_ig_ray_digest* trace,
                               hipStream_t s) {
    const void* k = (const void*)traj_union_kernel<WAVES, COUNT, TRACE>;
    // the all-ones word, pass_words words of the slice and the word of its clamp bit
    const size_t lds = ((size_t)pass_words + 2) * 4;
    static std::atomic<size_t> lds_set[64];
    const hipError_t e = allow_dynamic_lds(k, lds, lds_set, 64);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((traj_union_kernel<WAVES, COUNT, TRACE>), dim3(T), dim3(WAVES * 64), lds, s, m, c,
                       poses, L, boxes, pass_words, ig_union, counts, visits, trace);
    return hipGetLastError();
}

hipError_t launch_traj_union(int waves, const DevMap& m, const CamParams& c, const float* poses, uint32_t L,
                             uint32_t T, uint32_t pass_words, const TrajBox* boxes, float* ig_union,
                             uint32_t* counts, unsigned long long* visits, nbt_ig_ray_digest* trace,
                             hipStream_t s) {
    const bool count = visits != nullptr;    // no visit count when the caller does not ask for it
    const bool tr = trace != nullptr;
#define NBT_TU(W, C, R)                                                                              \
    if (waves == W && count == C && tr == R)                                                         \
        return launch_union<W, C, R>(m, c, poses, L, T, pass_words, boxes, ig_union, counts, visits, \
                                     trace, s);
    NBT_TU(4, true, false) NBT_TU(8, true, false) NBT_TU(16, true, false)
    NBT_TU(4, false, false) NBT_TU(8, false, false) NBT_TU(16, false, false)
    NBT_TU(4, true, true) NBT_TU(8, true, true) NBT_TU(16, true, true)
    NBT_TU(4, false, true) NBT_TU(8, false, true) NBT_TU(16, false, true)
#undef NBT_TU
    return hipErrorInvalidValue;
}

}  // namespace nbt
