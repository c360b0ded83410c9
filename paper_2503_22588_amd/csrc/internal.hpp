// internal.hpp -- types shared by the library's translation units (not installed).
#pragma once

#include <atomic>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nbt_ig.h"

namespace nbt {

// Encoded voxel word: the Eq. 2 gain of the voxel as float32 bits, with the
// sign bit set for Occupied voxels (their gain 1-P is still in the low 31
// bits).  The one-voxel border around the map holds kSentinel, the negative
// of the smallest denormal (2^-149): no gain takes it (1-P of an Occupied
// voxel is 0 or at least 2^-24), so a single signed test per step catches
// both "stop after this voxel" and "the walk left the map", and a walk that
// needs no visit count may add its magnitude instead of testing for it.
constexpr uint32_t kSentinel = 0x80000001u;
constexpr uint32_t kOccBit = 0x80000000u;
constexpr uint32_t kGainOne = 0x3F800000u;   // 1.0f: the gain of an Unknown voxel

// Storage order of the encoded words over the padded grid (X, Y, Z) =
// (x+1, y+1, z+1):
//   kLayoutLinear  x fastest: (Z*py + Y)*px + X;
//   column orders  T x T columns (T = 2, 4, 8): the x-y plane is cut into
//                  T x T tiles of T*T words (x fastest), each tile stores
//                  its layers z after z, and tiles go x fastest over the
//                  tile grid: ((Y/T*nbx + X/T)*pz + Z)*T*T + (Y%T)*T + X%T.
//                  For T = 4 a 128-B line holds a 4x4x2 block and four
//                  aligned layers a contiguous 4x4x4 block (256 B); a z step
//                  is always one layer.
// Padding of x and y up to whole tiles holds the sentinel as well.
constexpr int kLayoutLinear = NBT_IG_LAYOUT_LINEAR;

// log2 of the tile edge of a column order; 0 for the linear order.
__host__ __device__ inline int layout_tile_log2(int layout) {
    return layout == NBT_IG_LAYOUT_COLUMN2 ? 1
         : layout == NBT_IG_LAYOUT_COLUMN4 ? 2
         : layout == NBT_IG_LAYOUT_COLUMN8 ? 3 : 0;
}
inline bool valid_layout(int layout) { return layout >= NBT_IG_LAYOUT_LINEAR && layout <= NBT_IG_LAYOUT_COLUMN8; }

// Device view of an encoded map (passed to kernels by value).
struct DevMap {
    const uint32_t* enc;    // encoded words in `layout` order
    uint32_t bytes;         // size of enc in bytes (< 2^32)
    int nx, ny, nz;         // real dimensions
    int px, py, pz;         // padded dimensions (n + 2)
    int layout;             // NBT_IG_LAYOUT_*
    int tl;                 // log2 of the tile edge of a column order, 0 for the linear order
    int nbx, nby;           // tiles per axis over the padded x-y plane (column orders)
    float inv_s;            // 1/voxel_size (binary32)
    float ox, oy, oz;       // origin
};

// Byte offset of voxel (x, y, z), real coordinates in [-1, n] (the border
// included), in either layout.
__host__ __device__ inline uint32_t voxel_offset(const DevMap& m, int x, int y, int z) {
    const uint32_t X = (uint32_t)(x + 1), Y = (uint32_t)(y + 1), Z = (uint32_t)(z + 1);
    if (m.tl == 0) return ((Z * (uint32_t)m.py + Y) * (uint32_t)m.px + X) * 4u;
    const uint32_t t = (uint32_t)m.tl, lo = (1u << t) - 1u;
    const uint32_t tile = (Y >> t) * (uint32_t)m.nbx + (X >> t);
    return (((tile * (uint32_t)m.pz + Z) << (2u * t)) + ((Y & lo) << t | (X & lo))) * 4u;
}

// Endpoint-grid parameters derived once per launch on the host.
struct CamParams {
    int W, H;
    float dh, dv;           // range * tan(fov/2), binary32
    float range;
};

// Per-perspective reduction slot used when several workgroups share one
// perspective: fixed-point sums are order-independent, so the result is
// bit-identical whatever order the workgroups finish in.  The last
// workgroup of a perspective reads and clears its slot.
struct VpAccum {
    unsigned long long sum_fx;     // sum of ray gains * 2^24, rounded per workgroup
    unsigned long long steps;
    unsigned int count;            // workgroups done
    unsigned int invalid;
};
constexpr double kFixScale = 16777216.0;     // 2^24

// Launch shape of the viewpoint kernel.
struct VpLaunch {
    int waves;              // waves per workgroup (1, 2, 4, 8)
    int tile_w_log2;        // pixel tile of one wave: (1<<tile_w_log2) x (64>>tile_w_log2)
    int tiles_per_wave;     // tiles one wave walks per workgroup; 0 = balanced for the camera
    int xcd_remap;          // 0, or runs of this many consecutive workgroups per XCD
    int depth;              // gathers in flight per lane (1, 2, 4, 8)
};

// Voxel box of one trajectory's frusta (its bitset positions: x fastest).
struct TrajBox {
    int lx, ly, lz;          // min corner (voxels)
    int ax, ay, az;          // extent (voxels)
    uint32_t nbits;          // ax*ay*az, 0 for an empty trajectory
    uint32_t pad;
};

// ---- launchers (each defined next to its kernels) ----

hipError_t launch_encode_map(const float* prob, uint32_t* enc, const DevMap& m, float occ_thr,
                             float free_thr, unsigned int* bad_flag, hipStream_t s);
// Copies an encoded map into another storage order (dst laid out as dstm).
hipError_t launch_relayout(const DevMap& src, uint32_t* dst, const DevMap& dstm, hipStream_t s);

// trace != nullptr: the parity instance of the same kernel, which also writes
// one record per ray (trace[p * N_E + k]).
hipError_t launch_eval_viewpoints(const DevMap& m, const CamParams& c, const float* poses,
                                  uint32_t n, float* ig_out, unsigned long long* steps_out,
                                  VpAccum* ws, const VpLaunch& L, hipStream_t s,
                                  nbt_ig_ray_digest* trace = nullptr);

// Zeroes n per-perspective reduction slots (a fill kernel: no memset node
// when the caller captures the stream).
hipError_t launch_clear_slots(VpAccum* ws, uint32_t n, hipStream_t s);

hipError_t launch_trace_rays(const DevMap& m, const CamParams& c, const float* poses, uint32_t n,
                             nbt_ig_ray_digest* out, hipStream_t s);

hipError_t launch_trace_paths(const DevMap& m, const CamParams& c, const float* poses, uint32_t n,
                              const uint32_t* rays, uint32_t count, uint32_t max_len,
                              int32_t* lin_out, uint32_t* len_out, hipStream_t s);

hipError_t launch_traj_boxes(const DevMap& m, const CamParams& c, const float* poses, uint32_t T,
                             uint32_t L, TrajBox* boxes, hipStream_t s);

// Static LDS of the union kernel (its reductions); the bitset gets the rest.
size_t traj_static_lds_bytes();
// The timed union kernel of a workgroup size (4, 8, 16 waves), for occupancy queries.
const void* traj_union_kernel_ptr(int waves);

// One workgroup per trajectory, its bitset in LDS pass_words words at a time
// (boxes of more bits take several passes); trace != nullptr: the parity
// instance, one record per ray at trace[(t * L + l) * N_E + k].
hipError_t launch_traj_union(int waves, const DevMap& m, const CamParams& c, const float* poses, uint32_t L,
                             uint32_t T, uint32_t pass_words, const TrajBox* boxes, float* ig_union,
                             uint32_t* counts, unsigned long long* visits, nbt_ig_ray_digest* trace,
                             hipStream_t s);

// Kernel entry points of the persistent batched launch (for graph nodes).
const void* batch_kernel_ptr(int waves, int depth, bool count);
const void* batch_reset_ptr();

hipError_t launch_eval_cost(const float* id_pos, const float* id_ig, uint32_t nb, uint32_t np, float p,
                            const float* poses, uint32_t h, uint32_t k, const float poi[3], float tan_h,
                            float tan_v, float w_i, float eps, float* g_out, float* o_out, float* cost,
                            hipStream_t s);

// Number of workgroups a perspective is split into for a launch shape.
// Raises a kernel's dynamic-LDS limit to `bytes` on the current device when
// above the 64 KiB default, once per (kernel, device, size) seen; `cache`
// is the caller's per-kernel record of the largest size set per device.
inline hipError_t allow_dynamic_lds(const void* kernel, size_t bytes, std::atomic<size_t>* cache, int ncache) {
    if (bytes <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < ncache && cache[dev].load(std::memory_order_relaxed) >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess && dev >= 0 && dev < ncache) {
        size_t cur = cache[dev].load(std::memory_order_relaxed);
        while (cur < bytes && !cache[dev].compare_exchange_weak(cur, bytes)) {
        }
    }
    return e;
}

inline uint32_t vp_tiles(const CamParams& c, int tile_w_log2) {
    const int tw = 1 << tile_w_log2, th = 64 >> tile_w_log2;
    return (uint32_t)((c.W + tw - 1) / tw) * (uint32_t)((c.H + th - 1) / th);
}

// tiles_per_wave == 0: as few workgroups as 16 tiles per wave allow, with the
// tiles dealt evenly over them (no wave of a small camera left idle, no short
// last workgroup on a large one); when n perspectives (n > 0) would give
// fewer than 64 workgroups per CU, each perspective is split further (down to
// one tile per wave): small calls then fill the chip, and rays of uneven
// length (views that hit an object next to views into open space) spread
// over many short workgroups instead of a few long ones.
inline VpLaunch resolve_launch(const CamParams& c, VpLaunch L, uint32_t n = 0, int cu_count = 0) {
    if (L.tiles_per_wave > 0) return L;
    const uint32_t tiles = vp_tiles(c, L.tile_w_log2);
    const uint32_t waves = (uint32_t)L.waves;
    uint32_t groups = (tiles + waves * 16 - 1) / (waves * 16);
    const uint64_t want = 64ull * (uint64_t)(cu_count > 0 ? cu_count : 0);
    if (n > 0 && (uint64_t)n * groups < want) {
        const uint32_t most = (tiles + waves - 1) / waves;
        const uint64_t g = (want + n - 1) / n;
        groups = (uint32_t)(g < most ? g : most);
        if (groups < 1) groups = 1;
    }
    const uint32_t tpw = (tiles + waves * groups - 1) / (waves * groups);
    L.tiles_per_wave = (int)(tpw > 0 ? tpw : 1);
    return L;
}

inline uint32_t vp_groups(const CamParams& c, const VpLaunch& L0, uint32_t n = 0, int cu_count = 0) {
    const VpLaunch L = resolve_launch(c, L0, n, cu_count);
    const uint32_t per = (uint32_t)(L.waves * L.tiles_per_wave);
    return (vp_tiles(c, L.tile_w_log2) + per - 1) / per;
}

}  // namespace nbt
