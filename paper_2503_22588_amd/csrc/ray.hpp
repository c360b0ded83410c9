// ray.hpp -- per-lane ray generation and 3D-DDA state (device code).
//
// One lane owns one ray.  Set-up turns pixel (i, j) of a perspective into a
// voxel-unit segment O -> O + D clipped to the map (Sec. III, endpoint
// calculation), then into Amanatides-Woo traversal state.  Every operation
// is a single binary32 operation in a fixed order (the library is built
// with -ffp-contract=off, correctly rounded division and IEEE denormals), so
// the visited voxel sequence is a deterministic function of the inputs.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace nbt {

enum RayStatus : int { kRayOk = 0, kRayMiss = 1, kRayInvalid = 2 };

struct RayState {
    int ix, iy, iz;          // current voxel (real coordinates)
    int sx, sy, sz;          // step direction per axis (-1, 0, +1)
    float tx, ty, tz;        // parameter of the next face crossing per axis
    float dtx, dty, dtz;     // parameter distance between crossings per axis
    float t1;                // end of the clipped segment
};

__device__ __forceinline__ float sel_min(float a, float b) { return (b < a) ? b : a; }
__device__ __forceinline__ float sel_max(float a, float b) { return (b > a) ? b : a; }

// One axis of the slab clip.  Returns false when the ray runs parallel to
// this axis' faces outside the map.
__device__ __forceinline__ bool clip_axis(float O, float D, int n, float& t0, float& t1,
                                          float& inv, bool& parallel) {
    parallel = fabsf(D) < 0x1p-100f;
    if (parallel) {
        inv = 0.0f;
        return (O >= 0.0f) && (O < (float)n);
    }
    inv = 1.0f / D;
    const float tA = (0.0f - O) * inv;
    const float tB = ((float)n - O) * inv;
    t0 = sel_max(t0, sel_min(tA, tB));
    t1 = sel_min(t1, sel_max(tA, tB));
    return true;
}

__device__ __forceinline__ void init_axis(float O, float D, float t0, float inv, bool parallel,
                                          int n, int& idx, int& step, float& tmax, float& tdelta) {
    float f = floorf(O + t0 * D);
    f = sel_max(f, 0.0f);
    f = sel_min(f, (float)(n - 1));
    idx = (int)f;
    if (parallel) {
        step = 0;
        tmax = __builtin_inff();
        tdelta = __builtin_inff();
    } else {
        step = D > 0.0f ? 1 : -1;
        tdelta = fabsf(inv);
        tmax = ((float)(idx + (step > 0 ? 1 : 0)) - O) * inv;
    }
}

// Pixel of lane `lane` inside a (1 << tw_log2) x (64 >> tw_log2) tile: the
// lane bits are dealt alternately to x and y (x first) while both sides have
// bits left, so every aligned group of 4 lanes covers a 2 x 2 pixel block and
// every 16 lanes a 4 x 4 block (8 x 8 tiles).  Compact lane groups gather
// from fewer distinct cache lines than rows of 4 or 16 pixels.
__device__ __forceinline__ void tile_pixel(int lane, int tw_log2, int& lx, int& ly) {
    int x = 0, y = 0, bx = 0, by = 0;
    const int th_log2 = 6 - tw_log2;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const int bit = (lane >> b) & 1;
        const bool to_x = bx < tw_log2 && (by >= th_log2 || bx <= by);
        if (to_x) x |= bit << bx++;
        else y |= bit << by++;
    }
    lx = x;
    ly = y;
}

// pose: 12 floats (row-major R camera->world, then t).
__device__ __forceinline__ int setup_ray(const DevMap& m, const CamParams& c, const float* pose,
                                         int i, int j, RayState& r) {
    float u = 0.0f, v = 0.0f;
    if (c.W > 1) u = c.dh * ((float)(2 * i - (c.W - 1)) / (float)(c.W - 1));
    if (c.H > 1) v = c.dv * ((float)(2 * j - (c.H - 1)) / (float)(c.H - 1));

    const float org[3] = {m.ox, m.oy, m.oz};
    float O[3], D[3];
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float w = pose[3 * a + 0] * u;
        w = w + pose[3 * a + 1] * v;
        w = w + pose[3 * a + 2] * c.range;
        const float t = pose[9 + a];
        const float e = t + w;
        O[a] = (t - org[a]) * m.inv_s;
        const float E = (e - org[a]) * m.inv_s;
        D[a] = E - O[a];
        finite = finite && __builtin_isfinite(O[a]) && __builtin_isfinite(E) && __builtin_isfinite(D[a]);
    }
    if (!finite) return kRayInvalid;

    float t0 = 0.0f, t1 = 1.0f;
    float inv[3];
    bool par[3];
    const int n[3] = {m.nx, m.ny, m.nz};
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = clip_axis(O[a], D[a], n[a], t0, t1, inv[a], par[a]) && inside;
    if (!inside || t0 > t1) return kRayMiss;

    init_axis(O[0], D[0], t0, inv[0], par[0], n[0], r.ix, r.sx, r.tx, r.dtx);
    init_axis(O[1], D[1], t0, inv[1], par[1], n[1], r.iy, r.sy, r.ty, r.dty);
    init_axis(O[2], D[2], t0, inv[2], par[2], n[2], r.iz, r.sz, r.tz, r.dtz);
    r.t1 = t1;
    return kRayOk;
}

// Buffer resource over the encoded grid: out-of-range offsets read 0 instead
// of faulting, which keeps any indexing mistake inside the map's allocation.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t map_rsrc(const DevMap& m) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)m.enc, (short)0, (int)m.bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t load_word(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)byte_off, 0, 0);
}

__device__ __forceinline__ unsigned long long fnv1a_u32(unsigned long long h, uint32_t v) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        h ^= (unsigned long long)((v >> (8 * b)) & 0xFFu);
        h *= 0x100000001b3ULL;
    }
    return h;
}

constexpr unsigned long long kFnvBasis = 0xcbf29ce484222325ULL;

// Canonical linear index (z*ny + y)*nx + x of the voxel whose word sits at
// byte offset `off` of the encoded grid, in the map's storage order: the
// inverse of voxel_offset, written from the layout definitions rather than
// from the walk's per-axis deltas.  -1 for a border or padding word.
__device__ __forceinline__ int32_t offset_to_lin(const DevMap& m, uint32_t off) {
    const uint32_t w = off >> 2;
    uint32_t X, Y, Z;
    if (m.tl == 0) {
        X = w % (uint32_t)m.px;
        const uint32_t r = w / (uint32_t)m.px;
        Y = r % (uint32_t)m.py;
        Z = r / (uint32_t)m.py;
    } else {
        const uint32_t t = (uint32_t)m.tl, edge = 1u << t;
        const uint32_t in_tile = w & (edge * edge - 1u);
        const uint32_t r = w >> (2u * t);
        Z = r % (uint32_t)m.pz;
        const uint32_t tile = r / (uint32_t)m.pz;
        X = (tile % (uint32_t)m.nbx) * edge + (in_tile & (edge - 1u));
        Y = (tile / (uint32_t)m.nbx) * edge + (in_tile >> t);
    }
    const int x = (int)X - 1, y = (int)Y - 1, z = (int)Z - 1;
    if (x < 0 || y < 0 || z < 0 || x >= m.nx || y >= m.ny || z >= m.nz) return -1;
    return (z * m.ny + y) * m.nx + x;
}

// Parity mode of the throughput walks.  A walk instantiated with WalkTrace
// keeps, beside each gather in flight, the byte offset it was issued for and
// whether the generator was still inside the segment; every consumed visit
// is folded into the record from that offset (decoded by offset_to_lin), so
// the record shows the voxels the walk actually read, in its order.  Walks
// instantiated with NoTrace compile to the timed code.
struct NoTrace {};
struct WalkTrace {
    unsigned long long hash = kFnvBasis;   // FNV-1a-64 of the visited linear indices
    double gain = 0.0;                     // the visited words' gains, binary64 in visiting order
    uint32_t steps = 0;
    int32_t last = -1;                     // linear index of the last visit
    int reason = -1;                       // NBT_IG_RAY_*, -1 while walking
    uint32_t mismatch = 0;                 // union walk: visits whose bitset position names another voxel
    uint32_t box_bits = 0;                 // union walk: positions of the trajectory's box

    // slot consumed while the lane is still walking: word x read at `off`,
    // `live` = the generator had not passed the segment end when it issued it
    __device__ __forceinline__ void consume(const DevMap& m, uint32_t x, uint32_t off, bool live, float t1) {
        if (x != kSentinel) {
            const int32_t lin = offset_to_lin(m, off);
            hash = fnv1a_u32(hash, (uint32_t)lin);
            gain += (double)__uint_as_float(x & ~kOccBit);
            ++steps;
            last = lin;
        }
        if ((int)x < 0)
            reason = x != kSentinel ? NBT_IG_RAY_HIT
                   : live ? NBT_IG_RAY_EXIT : (t1 == 1.0f ? NBT_IG_RAY_END : NBT_IG_RAY_EXIT);
    }
    // end of the walk: a walk cut by its guard reports EXIT, as the reference walk does
    __device__ __forceinline__ void finish() {
        if (reason < 0) reason = NBT_IG_RAY_EXIT;
    }
};

template <class TR> constexpr bool traced() { return !std::is_same<TR, NoTrace>::value; }

// The parity record of one ray from its set-up status and walk record.
__device__ __forceinline__ void write_trace(nbt_ig_ray_digest* out, int status, const WalkTrace& rec) {
    nbt_ig_ray_digest d;
    d.hash = kFnvBasis;
    d.gain = 0.0;
    d.steps = 0;
    d.stop_lin = -1;
    d.reason = NBT_IG_RAY_MISS;
    d.reserved = 0;
    if (status == kRayInvalid) {
        d.reason = NBT_IG_RAY_INVALID;
        d.gain = __builtin_nan("");
    } else if (status == kRayOk) {
        d.hash = rec.hash;
        d.gain = rec.gain;
        d.steps = rec.steps;
        d.stop_lin = rec.last;
        d.reason = (uint32_t)rec.reason;
        d.reserved = rec.mismatch;
    }
    *out = d;
}

// Reason a walk stopped (matches NBT_IG_RAY_*).
enum WalkEnd : int { kEndHit = NBT_IG_RAY_HIT, kEndEnd = NBT_IG_RAY_END, kEndExit = NBT_IG_RAY_EXIT };

// Walks one ray.  Per visited voxel the encoded word is gathered and its gain
// added; the walk stops after an Occupied voxel, on the border sentinel (the
// previous voxel was the last), or when the next face crossing lies beyond
// the segment end.  The voxel coordinates are kept and addressed through
// voxel_offset (either layout); when TRACK is set visit(x, y, z, word) runs
// for every visited voxel.
template <bool TRACK, class Visit>
__device__ __forceinline__ int walk_ray(const DevMap& m, __amdgpu_buffer_rsrc_t rs, RayState& r,
                                        double& acc, uint32_t& steps, Visit&& visit) {
    const float dtx = r.dtx, dty = r.dty, dtz = r.dtz;
    float tx = r.tx, ty = r.ty, tz = r.tz;
    const float t1 = r.t1;
    const uint32_t guard = (uint32_t)(m.nx + m.ny + m.nz + 3);
    uint32_t n = 0;
    uint32_t bits;
    float tm;
    for (;;) {
        bits = load_word(rs, voxel_offset(m, r.ix, r.iy, r.iz));
        const bool sentinel = bits == kSentinel;
        const float g = sentinel ? 0.0f : __uint_as_float(bits & ~kOccBit);
        acc += (double)g;
        n += sentinel ? 0u : 1u;
        if constexpr (TRACK) {
            if (!sentinel) visit(r.ix, r.iy, r.iz, bits);
        }
        tm = fminf(fminf(tx, ty), tz);
        if ((int)bits < 0 || tm > t1 || n >= guard) break;
        const bool bx = (tx == tm);
        const bool by = !bx && (ty == tm);
        const bool bz = !bx && !by;
        const float nt = tm + (bx ? dtx : (by ? dty : dtz));
        tx = bx ? nt : tx;
        ty = by ? nt : ty;
        tz = bz ? nt : tz;
        r.ix += bx ? r.sx : 0;
        r.iy += by ? r.sy : 0;
        r.iz += bz ? r.sz : 0;
    }
    steps += n;
    if ((int)bits < 0) return bits == kSentinel ? kEndExit : kEndHit;
    if (tm > t1) return t1 == 1.0f ? kEndEnd : kEndExit;
    return kEndExit;
}

// Per-ray constants of the incremental map offset.  Linear layout: a step on
// axis a adds d[a] bytes.  Column orders (T x T tiles, T = 1 << TL): a z step
// adds dz (one layer of T*T words); an x or y step inside the tile adds dx or
// dy (the in-tile stride) and one across a tile face adds bigx or bigy.  The
// step crosses when the voxel's in-tile coordinate on that axis is T-1
// (forward) or 0 (backward), i.e. when ((off ^ flip) & mask) == 0, with the
// in-tile x and y in the fields tile_mask_x/y of the byte offset (TL bits
// each, from bit 2) and flip holding T-1 in the fields of the forward axes.
struct OffsetSteps {
    int dx, dy, dz;
    int bigx, bigy;
    uint32_t flip;
};

template <int TL> constexpr uint32_t tile_mask_x() { return ((1u << TL) - 1u) << 2; }
template <int TL> constexpr uint32_t tile_mask_y() { return ((1u << TL) - 1u) << (2 + TL); }

// TL: 0 for the linear order, else log2 of the column tile edge (m.tl).
template <int TL>
__device__ __forceinline__ OffsetSteps offset_steps(const DevMap& m, const RayState& r) {
    OffsetSteps o;
    if constexpr (TL == 0) {
        o.dx = r.sx * 4;
        o.dy = r.sy * m.px * 4;
        o.dz = r.sz * m.px * m.py * 4;
        o.bigx = o.bigy = 0;
        o.flip = 0;
    } else {
        constexpr int T = 1 << TL;
        constexpr int layer = 4 * T * T;       // bytes of one layer of a tile
        const int column = layer * m.pz;       // bytes of one tile's column
        o.dx = r.sx * 4;
        o.dy = r.sy * 4 * T;
        o.dz = r.sz * layer;
        o.bigx = r.sx * (column - 4 * (T - 1));
        o.bigy = r.sy * (column * m.nbx - 4 * T * (T - 1));
        o.flip = (r.sx > 0 ? tile_mask_x<TL>() : 0u) | (r.sy > 0 ? tile_mask_y<TL>() : 0u);
    }
    return o;
}

// One generator step of the pipelined walk: move to the next voxel unless
// the next face crossing lies beyond the segment end.  Past the end the
// generator points at offset 0, the sentinel word in the corner of the
// border (either layout), so every later gather reads "stop" without the
// loaded value ever being inspected here (which would force a wait for it).
// Loop invariants are passed by value so that the axis choice stays a
// register select.
template <int TL>
__device__ __forceinline__ void dda_advance(float& tx, float& ty, float& tz, uint32_t& off,
                                            bool& alive, float t1, int dxo, int dyo, int dzo,
                                            int bxo, int byo, uint32_t flip,
                                            float dtx, float dty, float dtz) {
    const float x = tx, y = ty, z = tz;
    const float tm = fminf(fminf(x, y), z);
    const bool go = alive && !(tm > t1);
    const bool ex = x == tm, ey = y == tm;
    const bool bx = go && ex;
    const bool by = go && !ex && ey;
    const bool bz = go && !ex && !ey;
    int d;
    if constexpr (TL != 0) {
        // x or y: the in-tile stride, or the tile-crossing delta at the tile
        // face; z: one layer.  Two selects fewer than a 3-axis edge test.
        const uint32_t msk = bx ? tile_mask_x<TL>() : tile_mask_y<TL>();
        const int big = bx ? bxo : byo;
        const int small = bx ? dxo : dyo;
        const int dxy = ((off ^ flip) & msk) == 0u ? big : small;
        d = bz ? dzo : dxy;
    } else {
        d = bx ? dxo : (by ? dyo : dzo);
    }
    off = go ? off + (uint32_t)d : 0u;
    // the stepping axis gains its delta, the others add +0 (t >= 0, so exact):
    // three selects and three adds instead of five selects and one add
    tx = x + (bx ? dtx : 0.0f);
    ty = y + (by ? dty : 0.0f);
    tz = z + (bz ? dtz : 0.0f);
    alive = go;
}

// Software-pipelined walk for the throughput kernels.  The voxel sequence of
// a ray depends only on its geometry, never on the map contents, so a
// generator runs P-1 voxels ahead of the consumer and keeps P gathers in
// flight per lane; the consumer adds gains in visiting order and stops at
// the first Occupied word or at a sentinel (the border, or the corner word
// the generator reads once the segment has ended).  Visits, gains and their
// order are exactly those of walk_ray (the sum is rounded differently, see
// below); only the reason is not reported, and the visit count only when
// COUNT is set.  Gathers past a stop are never
// consumed (and out-of-range ones read 0).  TL selects the map order (see offset_steps).
constexpr uint32_t kRunSlots = 8;

template <int P, bool COUNT, int TL, class TR = NoTrace>
__device__ __forceinline__ void walk_ray_pipelined(const DevMap& m, __amdgpu_buffer_rsrc_t rs,
                                                   const RayState& r, double& acc, uint32_t& steps,
                                                   TR* tr = nullptr) {
    static_assert(P == 2 || P == 4 || P == 8, "pipeline depth");
    const OffsetSteps o = offset_steps<TL>(m, r);
    const float dtx = r.dtx, dty = r.dty, dtz = r.dtz;
    const float t1 = r.t1;
    uint32_t off = voxel_offset(m, r.ix, r.iy, r.iz);
    float tx = r.tx, ty = r.ty, tz = r.tz;
    bool alive = true;     // the generator has not yet passed the segment end

    uint32_t w[P];
    // parity mode only: the offset of each gather in flight and whether the
    // generator was inside the segment when it issued it
    [[maybe_unused]] uint32_t wo[P];
    [[maybe_unused]] bool wl[P];
    w[0] = load_word(rs, off);
    if constexpr (traced<TR>()) {
        wo[0] = off;
        wl[0] = true;
    }
#pragma unroll
    for (int u = 1; u < P; ++u) {
        dda_advance<TL>(tx, ty, tz, off, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                           dtx, dty, dtz);
        w[u] = load_word(rs, off);
        if constexpr (traced<TR>()) {
            wo[u] = off;
            wl[u] = alive;
        }
    }
    uint32_t n = 0;
    // Every axis index moves one way only, so the border is reached within
    // nx + ny + nz steps; the group budget only guards that argument.
    uint32_t budget = (uint32_t)(m.nx + m.ny + m.nz + 3) / P + 2;
    bool run = true;
    // Gains are summed in binary32 over runs of kRunSlots consecutive slots and
    // each run's sum is added to the double accumulator.  The runs start at
    // fixed slot indices whatever P is, so every depth gives the same bits; a
    // sum of 8 non-negative terms is off by at most 7 units of 2^-24 relative.
    float part = 0.0f;
    uint32_t group = 0;
    // Lanes leave the loop between groups of P slots; inside a group every slot
    // runs for every lane still in the loop, with a lane that has stopped adding
    // nothing.  No slot is conditional, so slot u's word lives in one register
    // across iterations and each read waits only for its own gather (the P - 1
    // issued after it stay in flight).  A stopped lane issues at most P - 1
    // spare gathers before it leaves.
    while (run) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const uint32_t x = w[u];
            // a voxel visit, not the sentinel.  The IG-only walk skips the test:
            // the sentinel then adds its magnitude 2^-149, at most once per ray
            // (it stops the walk), so a ray sum and the IG are off by at most
            // 2^-149 absolute.
            const bool take = COUNT ? (run && x != kSentinel) : run;
            // the empty asm keeps each slot's read ahead of its refill (else the
            // reads sink to the end of the group and the refills need copies)
            uint32_t xs = take ? x : 0u;
            asm volatile("" : "+v"(xs));
            part += fabsf(__uint_as_float(xs));
            if constexpr (COUNT) n += take ? 1u : 0u;
            if constexpr (traced<TR>()) {
                if (run) tr->consume(m, x, wo[u], wl[u], t1);
            }
            run = run && (int)x >= 0;
            dda_advance<TL>(tx, ty, tz, off, alive, t1, o.dx, o.dy, o.dz, o.bigx, o.bigy, o.flip,
                               dtx, dty, dtz);
            w[u] = load_word(rs, off);
            if constexpr (traced<TR>()) {
                wo[u] = off;
                wl[u] = alive;
            }
        }
        if ((++group & (kRunSlots / P - 1)) == 0u) {
            acc += (double)part;
            part = 0.0f;
        }
        run = run && --budget != 0u;
    }
    acc += (double)part;
    if constexpr (COUNT) steps += n;
    if constexpr (traced<TR>()) tr->finish();
}

}  // namespace nbt
