// surrogate.hip -- learned IG surrogate: patch, conv3d trunk and MLP on BF16
// MFMA (FP32 accumulation), radix selection of the candidates to rescore (also
// the generic top-k) and the final pick after exact rescoring.
//
// The trunk's fragments follow v_mfma_f32_16x16x32_bf16 (gfx950): for lane
// l, A (16 x 32) row l%16 holds k = (l/16)*8 .. +7, B (32 x 16) column l%16
// holds the same k, and the 16 x 16 result gives lane l column l%16, rows
// (l/16)*4 .. +3.  The MLP uses the 32 x 32 forms (see there).
#include "internal.hpp"
#include "ray.hpp"
#include "surrogate.hpp"

namespace nbt {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4_t mfma16(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- patch ----
// Occupied and unknown voxel counts over each cell's f^3 voxels (voxels
// outside the map count as neither), divided by f^3.  One workgroup per run
// of kPatchRun cells along x; its threads take the run's rows of f voxels
// along x (cell fastest, then y, then z, so a wave reads contiguous runs of
// the map) and add their counts in LDS.
constexpr int kPatchRun = 8;

__global__ __launch_bounds__(256) void patch_kernel(DevMap m, int f, int i0x, int i0y, int i0z,
                                                    __bf16* __restrict__ out_bf16,
                                                    float* __restrict__ out_f32) {
    __shared__ uint32_t s_occ[kPatchRun], s_unk[kPatchRun];
    const int cell0 = (int)blockIdx.x * kPatchRun;
    const int cx0 = cell0 % kGrid, cy = (cell0 / kGrid) % kGrid, cz = cell0 / (kGrid * kGrid);
    if (threadIdx.x < kPatchRun) s_occ[threadIdx.x] = s_unk[threadIdx.x] = 0u;
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);
    const int rows = kPatchRun * f * f;
    for (int it = (int)threadIdx.x; it < rows; it += (int)blockDim.x) {
        const int c = it % kPatchRun, r = it / kPatchRun;
        const int y = i0y + cy * f + r % f, z = i0z + cz * f + r / f;
        if (y < 0 || y >= m.ny || z < 0 || z >= m.nz) continue;
        const int x0 = i0x + (cx0 + c) * f;
        uint32_t occ = 0, unk = 0;
#pragma unroll 4
        for (int dx = 0; dx < f; ++dx) {
            const int x = x0 + dx;
            const uint32_t w = (x >= 0 && x < m.nx) ? load_word(rs, voxel_offset(m, x, y, z)) : 0u;
            occ += (w & kOccBit) ? 1u : 0u;
            unk += (w == kGainOne) ? 1u : 0u;
        }
        if (occ) atomicAdd(&s_occ[c], occ);
        if (unk) atomicAdd(&s_unk[c], unk);
    }
    __syncthreads();
    if (threadIdx.x < kPatchRun) {
        const int cell = cell0 + (int)threadIdx.x;
        const float vol = (float)((double)f * f * f);
        const float fo = (float)s_occ[threadIdx.x] / vol, fu = (float)s_unk[threadIdx.x] / vol;
        if (out_bf16) {
            out_bf16[cell] = (__bf16)fo;
            out_bf16[kPatchCells + cell] = (__bf16)fu;
        }
        if (out_f32) {
            out_f32[cell] = fo;
            out_f32[kPatchCells + cell] = fu;
        }
    }
}

// ---------------------------------------------------------------- trunk ----
// The trunk in four launches (after the patch pass for wide cells, below).
// trunk_front: workgroup b of 64 owns a 2^3 block of the 8^3 conv2 outputs.
// It takes the 11^3 patch cells that block depends on (cells outside the
// 32^3 patch are conv1's zero padding) into LDS as BF16 fractions: counted
// straight from the map, one thread per cell, when cells are at most
// kFrontCountMaxF voxels wide, else read from the patch that launch_patch
// counted over the whole chip first (64 workgroups counting 5^3-voxel cells
// took 74 us; the separate pass spreads them over every CU).
// It then computes the 5^3 conv1
// outputs around its block (those outside the 16^3 grid are conv2's zero
// padding) and its eight conv2 positions, all from LDS, and stores them
// channel-last, [z][y][x][32].  conv3, conv4 and the pose-independent part
// of fc1 follow as three small launches that split each layer's weights
// (the bulk of what the tail reads) over 4, 4 and 16 workgroups.  Kernel
// boundaries order the steps: a device-scope fence in every workgroup would
// write back and invalidate its XCD's L2 instead.
//
// conv2..conv4 are implicit GEMMs whose reduction index is tap-major,
// k = tap * cin + ci (tap = (dz*3 + dy)*3 + dx), so that the 8 consecutive k
// of one lane's MFMA fragment are 8 consecutive channels of one input voxel:
// one 16-byte load from the channel-last activations.  The weights are
// stored in that order, zero-padded to whole 32-wide k chunks.
constexpr int kTrunkThreads = 1024;
constexpr int kCells = 11;                        // patch cells per axis a block depends on
constexpr int kCells3 = kCells * kCells * kCells;
constexpr int kC1 = 5;                            // conv1 outputs per axis a block computes

__device__ __forceinline__ bf16x8_t bf16_zero8() {
    bf16x8_t z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ __bf16 relu_bf16(float v) { return (__bf16)(v > 0.0f ? v : 0.0f); }

__device__ __forceinline__ void tap_dxyz(int tap, int& dz, int& dy, int& dx) {
    dz = tap / 9;
    dy = (tap / 3) % 3;
    dx = tap % 3;
}

// The 11^3 patch cells 8b-3 .. 8b+7 (per axis) that block b depends on, as
// BF16 fractions in `patch`: counted from the map, one thread per cell (F
// voxels per cell and axis), or read from the counted patch p.patch.
template <int F>
__device__ __forceinline__ void front_cells(const TrunkArgs& p, int bx, int by, int bz,
                                            __bf16 (&patch)[2][kCells3]) {
    const int cx0 = 8 * bx - 3, cy0 = 8 * by - 3, cz0 = 8 * bz - 3;
    const DevMap& m = p.m;
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);
    for (int cell = threadIdx.x; cell < kCells3; cell += kTrunkThreads) {
        const int clx = cell % kCells, cly = (cell / kCells) % kCells, clz = cell / (kCells * kCells);
        const int cx = cx0 + clx, cy = cy0 + cly, cz = cz0 + clz;
        __bf16 fo = (__bf16)0.0f, fu = (__bf16)0.0f;
        if ((unsigned)cx < (unsigned)kGrid && (unsigned)cy < (unsigned)kGrid && (unsigned)cz < (unsigned)kGrid) {
            if constexpr (F == 0) {
                const int pc = (cz * kGrid + cy) * kGrid + cx;
                fo = p.patch[pc];
                fu = p.patch[kPatchCells + pc];
            } else {
                const int x0 = p.i0x + cx * F, y0 = p.i0y + cy * F, z0 = p.i0z + cz * F;
                uint32_t occ = 0, unk = 0;
#pragma unroll
                for (int dz = 0; dz < F; ++dz) {
#pragma unroll
                    for (int dy = 0; dy < F; ++dy) {
                        const int y = y0 + dy, z = z0 + dz;
                        const bool yz = y >= 0 && y < m.ny && z >= 0 && z < m.nz;
#pragma unroll
                        for (int dx = 0; dx < F; ++dx) {
                            const int x = x0 + dx;
                            const uint32_t w =
                                (yz && x >= 0 && x < m.nx) ? load_word(rs, voxel_offset(m, x, y, z)) : 0u;
                            occ += (w & kOccBit) ? 1u : 0u;
                            unk += (w == kGainOne) ? 1u : 0u;
                        }
                    }
                }
                const float vol = (float)(F * F * F);
                fo = (__bf16)((float)occ / vol);
                fu = (__bf16)((float)unk / vol);
            }
        }
        patch[0][cell] = fo;
        patch[1][cell] = fu;
    }
}

__global__ __launch_bounds__(kTrunkThreads) void trunk_front_kernel(TrunkArgs p) {
    __shared__ __bf16 s_patch[2][kCells3];
    __shared__ __align__(16) __bf16 s_act1[kC1 * kC1 * kC1 * 16];
    __shared__ f32x4_t s_part[8][64];

    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63, row = lane & 15, kq = lane >> 4;
    const int bx = blockIdx.x & 3, by = (blockIdx.x >> 2) & 3, bz = blockIdx.x >> 4;

    // ---- patch cells 8b-3 .. 8b+7 per axis ----
    static_assert(kFrontCountMaxF == 2, "the front counts cells of 1 or 2 voxels");
    if (p.patch) front_cells<0>(p, bx, by, bz, s_patch);
    else if (p.f == 1) front_cells<1>(p, bx, by, bz, s_patch);
    else front_cells<2>(p, bx, by, bz, s_patch);
    __syncthreads();

    // ---- conv1 outputs 4b-1 .. 4b+3 per axis (125 positions x 16 channels) ----
    // k = ci*27 + tap (54, padded to 64); positions outside 0..15 are stored as 0
    if (wave < 8) {
        const int ml = wave * 16 + row;                                  // A row: local position
        const int lz = ml / 25, ly = (ml / 5) % 5, lx = ml % 5;
        f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            bf16x8_t a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = ch * 32 + kq * 8 + e;
                __bf16 v = (__bf16)0.0f;
                if (k < 54 && ml < kC1 * kC1 * kC1) {
                    const int ci = k / 27;
                    int dz, dy, dx;
                    tap_dxyz(k - ci * 27, dz, dy, dx);
                    v = s_patch[ci][((2 * lz + dz) * kCells + (2 * ly + dy)) * kCells + 2 * lx + dx];
                }
                a[e] = v;
            }
            const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(p.w[0] + row * 64 + ch * 32 + kq * 8);
            acc = mfma16(a, b, acc);
        }
        const float bias = p.b[0][row];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mo = wave * 16 + kq * 4 + r;
            if (mo < kC1 * kC1 * kC1) {
                const int oz = 4 * bz - 1 + mo / 25, oy = 4 * by - 1 + (mo / 5) % 5, ox = 4 * bx - 1 + mo % 5;
                const bool inside = (unsigned)oz < 16u && (unsigned)oy < 16u && (unsigned)ox < 16u;
                s_act1[mo * 16 + row] = inside ? relu_bf16(acc[r] + bias) : (__bf16)0.0f;
            }
        }
    }
    __syncthreads();

    // ---- conv2 outputs 2b .. 2b+1 per axis (8 positions x 32 channels) ----
    // k = tap*16 + ci (432, padded to 448: 14 chunks); wave w: column tile w & 1,
    // chunks w/2, w/2 + 4, ...; the four partial tiles added in a fixed order
    if (wave < 8) {
        const int nt = wave & 1, part = wave >> 1;
        const int z = (row >> 2) & 1, y = (row >> 1) & 1, x = row & 1;      // rows 8..15 unused
        f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const __bf16* wr = p.w[1] + (nt * 16 + row) * 448 + kq * 8;
#pragma unroll
        for (int ch = part; ch < 14; ch += 4) {
            const int tap = 2 * ch + (kq >> 1), c0 = (kq & 1) * 8;
            bf16x8_t a = bf16_zero8();
            if (tap < 27 && row < 8) {
                int dz, dy, dx;
                tap_dxyz(tap, dz, dy, dx);
                a = *reinterpret_cast<const bf16x8_t*>(
                    s_act1 + (((2 * z + dz) * kC1 + (2 * y + dy)) * kC1 + 2 * x + dx) * 16 + c0);
            }
            const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(wr + ch * 32);
            acc = mfma16(a, b, acc);
        }
        s_part[wave][lane] = acc;
    }
    __syncthreads();
    if (wave < 2) {
        const f32x4_t acc = ((s_part[wave][lane] + s_part[wave + 2][lane]) + s_part[wave + 4][lane]) +
                            s_part[wave + 6][lane];
        const int n = wave * 16 + row;
        const float bias = p.b[1][n];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mo = kq * 4 + r;
            if (mo < 8) {
                const int oz = 2 * bz + (mo >> 2), oy = 2 * by + ((mo >> 1) & 1), ox = 2 * bx + (mo & 1);
                p.act2[((oz * 8 + oy) * 8 + ox) * 32 + n] = relu_bf16(acc[r] + bias);
            }
        }
    }

}

// conv3: 8^3 x 32 -> 4^3 x 64, k = tap*32 + ci (864).  Workgroup j owns output
// channels 16j..16j+15 (its weights, 27 KiB, are read by it alone), wave w
// the positions 16w..16w+15; conv2's output is staged in LDS.
__global__ __launch_bounds__(256) void trunk_conv3_kernel(TrunkArgs p) {
    __shared__ __align__(16) __bf16 s_act2[512 * 32];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63, row = lane & 15, kq = lane >> 4;
    const int nt = blockIdx.x;
    bf16x8_t b3[27];                                  // requested before the staging
    {
        const __bf16* wr = p.w[2] + (nt * 16 + row) * 864 + kq * 8;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) b3[tap] = *reinterpret_cast<const bf16x8_t*>(wr + tap * 32);
    }
    {
        bf16x8_t piece[8];                            // all requested before the first LDS write
#pragma unroll
        for (int j = 0; j < 8; ++j) piece[j] = reinterpret_cast<const bf16x8_t*>(p.act2)[t + 256 * j];
#pragma unroll
        for (int j = 0; j < 8; ++j) reinterpret_cast<bf16x8_t*>(s_act2)[t + 256 * j] = piece[j];
    }
    __syncthreads();
    const int mm = wave * 16 + row;
    const int z = mm >> 4, y = (mm >> 2) & 3, x = mm & 3;
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
        int dz, dy, dx;
        tap_dxyz(tap, dz, dy, dx);
        const int iz = 2 * z + dz - 1, iy = 2 * y + dy - 1, ix = 2 * x + dx - 1;
        bf16x8_t a = bf16_zero8();
        if ((unsigned)iz < 8u && (unsigned)iy < 8u && (unsigned)ix < 8u)
            a = *reinterpret_cast<const bf16x8_t*>(s_act2 + ((iz * 8 + iy) * 8 + ix) * 32 + kq * 8);
        acc = mfma16(a, b3[tap], acc);
    }
    const int n = nt * 16 + row;
    const float bias = p.b[2][n];
#pragma unroll
    for (int r = 0; r < 4; ++r) p.act3[(wave * 16 + kq * 4 + r) * 64 + n] = relu_bf16(acc[r] + bias);
}

// conv4: 4^3 x 64 -> 2^3 x 64, k = tap*64 + ci (1728).  Workgroup j owns
// output channels 16j..16j+15; its four waves split the 54 k chunks and add
// their partial tiles in a fixed order.  Writes the 512 features (BF16),
// index c*8 + z*4 + y*2 + x.
__global__ __launch_bounds__(256) void trunk_conv4_kernel(TrunkArgs p) {
    __shared__ __align__(16) __bf16 s_act3[64 * 64];
    __shared__ f32x4_t s_part[4][64];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63, row = lane & 15, kq = lane >> 4;
    const int nt = blockIdx.x;
    bf16x8_t b4[14];                                  // chunks wave, wave + 4, ...
    {
        const __bf16* wr = p.w[3] + (nt * 16 + row) * 1728 + kq * 8;
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            const int ch = wave + 4 * i;
            b4[i] = ch < 54 ? *reinterpret_cast<const bf16x8_t*>(wr + ch * 32) : bf16_zero8();
        }
    }
    {
        const bf16x8_t a0 = reinterpret_cast<const bf16x8_t*>(p.act3)[t];
        const bf16x8_t a1 = reinterpret_cast<const bf16x8_t*>(p.act3)[t + 256];
        reinterpret_cast<bf16x8_t*>(s_act3)[t] = a0;
        reinterpret_cast<bf16x8_t*>(s_act3)[t + 256] = a1;
    }
    __syncthreads();
    const int z = (row >> 2) & 1, y = (row >> 1) & 1, x = row & 1;      // rows 8..15 unused
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < 14; ++i) {
        const int ch = wave + 4 * i;
        if (ch < 54) {
            const int tap = ch >> 1, c0 = (ch & 1) * 32 + kq * 8;
            int dz, dy, dx;
            tap_dxyz(tap, dz, dy, dx);
            const int iz = 2 * z + dz - 1, iy = 2 * y + dy - 1, ix = 2 * x + dx - 1;
            bf16x8_t a = bf16_zero8();
            if (row < 8 && (unsigned)iz < 4u && (unsigned)iy < 4u && (unsigned)ix < 4u)
                a = *reinterpret_cast<const bf16x8_t*>(s_act3 + ((iz * 4 + iy) * 4 + ix) * 64 + c0);
            acc = mfma16(a, b4[i], acc);
        }
    }
    s_part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
        const f32x4_t sum = ((s_part[0][lane] + s_part[1][lane]) + s_part[2][lane]) + s_part[3][lane];
        const int n = nt * 16 + row;
        const float bias = p.b[3][n];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mo = kq * 4 + r;                // position z*4 + y*2 + x
            if (mo < 8) p.feat[n * 8 + mo] = relu_bf16(sum[r] + bias);
        }
    }
}

// c[n] = b1[n] + sum_k W1f[n][k] f[k] (the pose-independent part of fc1):
// workgroup j owns outputs 16j..16j+15, sixteen lanes per output with 32 k
// each, added by a fixed butterfly.
__global__ __launch_bounds__(256) void trunk_fc1_kernel(TrunkArgs p) {
    const int t = threadIdx.x;
    const int n = blockIdx.x * 16 + (t >> 4), q = t & 15;
    const __bf16* wr = p.w1f + (size_t)n * kFeat + q * 32;
    bf16x8_t w[4], f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w[i] = *reinterpret_cast<const bf16x8_t*>(wr + 8 * i);
        f[i] = *reinterpret_cast<const bf16x8_t*>(p.feat + q * 32 + 8 * i);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 8; ++e) s += (float)w[i][e] * (float)f[i][e];
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
    if (q == 0) p.c[n] = p.fb1[n] + s;
}

// ---------------------------------------------------------------- MLP ------
// Per pose: h1 = ReLU(c + W1d [u, dn]) (FP32, stored BF16), h2 = ReLU(W2 h1 +
// b2) (BF16 products, FP32 sums), y = out_scale * (W3 . h2 + b3).  One
// workgroup of 8 waves per CU holds W2 (rows padded to 264 halves), W1d, c, b2
// and W3 in LDS; each wave takes 32 poses at a time and computes h2 transposed
// (outputs x poses) on v_mfma_f32_32x32x16_bf16, which from one wave issues at
// about twice the rate of the 16x16x32 form per unit of work:
//   * A = a W2 fragment: lane l holds output row l%32 of the tile and 8
//     consecutive stored k positions (l/32)*8 .. +7 (one 16-byte LDS read);
//   * B = h1 transposed: lane l holds pose l%32 and the same 8 k positions;
//   * the 32 x 32 result gives lane l pose l%32 and outputs 8j + 4(l/32) + r
//     (j, r = 0..3) at element 4j + r.
// h1 comes from two chained v_mfma_f32_32x32x2_f32 per 32 neurons (neurons x
// poses, K = the four inputs u0 u1 u2 dn, c as the accumulator input): its
// result gives lane l pose l%32 and neurons 8j + 4(l/32) + r, which are the B
// elements of two k-steps once W2's stored k order swaps bits 2 and 3 of the
// index within each 16 (position q of a k-step holds neuron
// 8((q>>2)&1) + 4(q>>3) + (q&3)).  fc3 sums each lane's outputs and one
// exchange between the lane halves completes it.
constexpr int kW2Stride = kHidden + 8;
constexpr int kMlpWaves = 8;
// W1d transposed in LDS (input-major), rows padded so that the two lane
// halves reading inputs f and f+1 of 32 neurons hit different banks
constexpr int kW1dStride = kHidden + 32;
constexpr size_t kMlpLds =
    (size_t)kHidden * kW2Stride * sizeof(__bf16) + (size_t)(4 * kW1dStride + 3 * kHidden) * sizeof(float);
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// Rank key of a value: larger values give larger keys, -0 and +0 the same
// key, NaN the smallest.
__device__ __forceinline__ uint32_t mono_key(float v) {
    const uint32_t b = __float_as_uint(v);
    if (v != v) return 0u;
    if (v == 0.0f) return 0x80000000u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ __launch_bounds__(kMlpWaves * 64) void mlp_kernel(const float* __restrict__ poses, uint32_t n,
                                                             float px, float py, float pz, float dist_mean,
                                                             float dist_scale, const float* __restrict__ c,
                                                             const float* __restrict__ w1d,
                                                             const __bf16* __restrict__ w2,
                                                             const float* __restrict__ b2,
                                                             const float* __restrict__ w3, float b3,
                                                             float out_scale, float* __restrict__ pred) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* sw2 = reinterpret_cast<__bf16*>(smem);
    float* sw1d = reinterpret_cast<float*>(smem + (size_t)kHidden * kW2Stride * sizeof(__bf16));
    float* sc = sw1d + 4 * kW1dStride;
    float* sb2 = sc + kHidden;
    float* sw3 = sb2 + kHidden;
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, half = lane >> 5;
    const uint32_t ngroup = (n + 31) / 32;
    const uint32_t wave_global = blockIdx.x * kMlpWaves + (threadIdx.x >> 6);
    const uint32_t waves = gridDim.x * kMlpWaves;
    // this lane's first camera centre (pose col of the wave's first group),
    // requested before the LDS fill so that its latency passes during it
    float cen[3];
    {
        const uint32_t p = wave_global * 32 + col;
#pragma unroll
        for (int a = 0; a < 3; ++a) cen[a] = (wave_global < ngroup && p < n) ? poses[12 * (size_t)p + 9 + a] : 0.0f;
    }
    {
        // all 16 pieces of this thread requested before the first LDS write (a
        // load-wait-store loop would pay one memory round trip per piece)
        constexpr int kPer = kHidden * kHidden / 8 / (kMlpWaves * 64);
        bf16x8_t piece[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            piece[j] = reinterpret_cast<const bf16x8_t*>(w2)[threadIdx.x + j * kMlpWaves * 64];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = threadIdx.x + j * kMlpWaves * 64;
            const int r = (i * 8) / kHidden, k = (i * 8) % kHidden;
            *reinterpret_cast<bf16x8_t*>(sw2 + r * kW2Stride + k) = piece[j];
        }
    }
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        const f32x4_t w = *reinterpret_cast<const f32x4_t*>(w1d + 4 * i);
#pragma unroll
        for (int f = 0; f < 4; ++f) sw1d[f * kW1dStride + i] = w[f];
        sc[i] = c[i];
        sb2[i] = b2[i];
        sw3[i] = w3[i];
    }
    __syncthreads();

    for (uint32_t g = wave_global; g < ngroup; g += waves) {
        const uint32_t pose = g * 32 + col;
        float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f, dn = 0.0f;
        if (pose < n) {
            const float vx = cen[0] - px;
            const float vy = cen[1] - py;
            const float vz = cen[2] - pz;
            const float d = sqrtf(vx * vx + vy * vy + vz * vz);
            const float inv = d > 0.0f ? 1.0f / d : 0.0f;
            u0 = vx * inv;
            u1 = vy * inv;
            u2 = vz * inv;
            dn = (d - dist_mean) / dist_scale;
        }
        {
            const uint32_t g2 = g + waves;            // the next group's centre, if any
            const uint32_t p = g2 * 32 + col;
#pragma unroll
            for (int a = 0; a < 3; ++a) cen[a] = (g2 < ngroup && p < n) ? poses[12 * (size_t)p + 9 + a] : 0.0f;
        }
        // B operands of the two h1 products: inputs (u0, u1), then (u2, dn),
        // input `half` of each pair in this lane
        const float fin0 = half ? u1 : u0, fin1 = half ? dn : u2;
        f32x16_t acc[kHidden / 32];
#pragma unroll
        for (int t = 0; t < kHidden / 32; ++t)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
#pragma unroll 1
        for (int blk = 0; blk < kHidden / 32; ++blk) {
            // h1 of neurons 32 blk .. +31 for the wave's 32 poses
            f32x16_t h;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const f32x4_t cv = *reinterpret_cast<const f32x4_t*>(sc + 32 * blk + 8 * j + 4 * half);
#pragma unroll
                for (int r = 0; r < 4; ++r) h[4 * j + r] = cv[r];
            }
            const float wa0 = sw1d[half * kW1dStride + 32 * blk + col];
            const float wa1 = sw1d[(2 + half) * kW1dStride + 32 * blk + col];
            h = __builtin_amdgcn_mfma_f32_32x32x2f32(wa0, fin0, h, 0, 0, 0);
            h = __builtin_amdgcn_mfma_f32_32x32x2f32(wa1, fin1, h, 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // k-step 2 blk + t: elements 8t .. 8t+7 of h, ReLU, BF16
                bf16x8_t hb;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float v = h[8 * t + e];
                    hb[e] = (__bf16)(v > 0.0f ? v : 0.0f);
                }
                const __bf16* ak = sw2 + col * kW2Stride + (2 * blk + t) * 16 + half * 8;
#pragma unroll
                for (int ot = 0; ot < kHidden / 32; ++ot) {
                    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(ak + ot * 32 * kW2Stride);
                    acc[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hb, acc[ot], 0, 0, 0);
                }
            }
        }
        // fc3: this lane's outputs 32 ot + 8j + 4 half + r of pose `col`
        float part = 0.0f;
#pragma unroll
        for (int ot = 0; ot < kHidden / 32; ++ot) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = 32 * ot + 8 * j + 4 * half;
                const f32x4_t bb = *reinterpret_cast<const f32x4_t*>(sb2 + o);
                const f32x4_t ww = *reinterpret_cast<const f32x4_t*>(sw3 + o);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float h2 = acc[ot][4 * j + r] + bb[r];
                    part = __builtin_fmaf(ww[r], h2 > 0.0f ? h2 : 0.0f, part);
                }
            }
            __builtin_amdgcn_sched_barrier(0);    // one tile's b2 / W3 reads at a time
        }
        part += __shfl_xor(part, 32, 64);
        if (half == 0 && pose < n) pred[pose] = out_scale * (part + b3);
    }
}

// ------------------------------------------------------- radix selection ----
// The k largest of n predictions (ties to the lower index) as a set, with
// their poses for the exact rescoring, in stages of one 1024-thread
// workgroup per slice of items.  A workgroup holds its items in registers
// (R per thread) and finds the exact k-th rank key by histogram digits of 12
// bits of the key, from the highest bit in which its keys differ down, each
// over the items still tied with the bins chosen so far, and stops when the
// bin holding the k-th key is taken whole; of the keys equal to the k-th
// key it takes the lowest indices, found by two histograms of index bits
// when more are equal than needed.  Stage workgroups keep the k best of 4096 items each; the
// last stage (one workgroup, at most 16,384 items) writes the chosen
// candidates and copies their poses.  Sets are written in no particular
// order: the final pick after rescoring orders by exact IG and index.
constexpr int kSelThreads = 1024;
constexpr uint32_t kNoItem = 0xFFFFFFFFu;         // index of an empty slot
constexpr uint32_t kStageSlice = 4096;            // items per stage workgroup (4 per thread)
constexpr uint32_t kFinalItems = 16384;           // items of the last stage (16 per thread)

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSelThreads / 64; ++w) {
        const uint32_t s = s_wave[w];
        base += (w < wave) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// Bins 4t..4t+3 of s_hist (`bins` of them) per thread; the histogram is left
// zero.  DESC: the bin d with (items in bins above d) < need <= (items in
// bins d and above); otherwise counted from the lowest bin.  Returns d; sets
// beyond = the items strictly beyond d, in_bin = the items in d, total.
template <bool DESC>
__device__ __forceinline__ uint32_t find_bin(uint32_t* s_hist, uint32_t bins, uint32_t need, uint32_t* s_wave,
                                             uint32_t* s_out, uint32_t& beyond, uint32_t& in_bin,
                                             uint32_t& total) {
    uint32_t h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = 4 * threadIdx.x + q < bins ? s_hist[4 * threadIdx.x + q] : 0u;
    const uint32_t v = h[0] + h[1] + h[2] + h[3];
    const uint32_t ex = block_excl_scan(v, s_wave, total);     // (its barriers order the reads above)
    for (uint32_t i = threadIdx.x; i < bins; i += kSelThreads) s_hist[i] = 0u;
    uint32_t run = DESC ? total - ex - v : ex;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = DESC ? 3 - i : i;
        if (run < need && run + h[q] >= need) {
            s_out[0] = 4u * threadIdx.x + q;
            s_out[1] = run;
            s_out[2] = h[q];
        }
        run += h[q];
    }
    __syncthreads();
    const uint32_t d = s_out[0];
    beyond = s_out[1];
    in_bin = s_out[2];
    __syncthreads();
    return d;
}

// Max, min and count of the valid items' keys over the workgroup.
template <int R>
__device__ __forceinline__ void block_key_range(const uint32_t (&key)[R], const uint32_t (&idx)[R], uint32_t* s_red,
                                                uint32_t& kmax, uint32_t& kmin, uint32_t& count) {
    uint32_t mx = 0u, mn = 0xFFFFFFFFu, c = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (idx[r] != kNoItem) {
            mx = max(mx, key[r]);
            mn = min(mn, key[r]);
            ++c;
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
        mn = min(mn, (uint32_t)__shfl_xor(mn, o, 64));
        c += __shfl_xor(c, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_red[3 * wave] = mx;
        s_red[3 * wave + 1] = mn;
        s_red[3 * wave + 2] = c;
    }
    __syncthreads();
    kmax = 0u;
    kmin = 0xFFFFFFFFu;
    count = 0u;
#pragma unroll
    for (int w = 0; w < kSelThreads / 64; ++w) {
        kmax = max(kmax, s_red[3 * w]);
        kmin = min(kmin, s_red[3 * w + 1]);
        count += s_red[3 * w + 2];
    }
    __syncthreads();
}

// Calls emit(key, idx) once for each of the k best valid items the workgroup
// holds (all of them when there are at most k).  The key digits start below
// the bits all valid keys share (found from their max and min), 12 bits at a
// time, so that the first histogram is spread over the keys' actual range;
// as soon as the bin holding the k-th key is taken whole, the items with a
// digit prefix at or above it are the k best and no further pass is made.
template <int R, class EMIT>
__device__ __forceinline__ void block_select(const uint32_t (&key)[R], const uint32_t (&idx)[R], uint32_t k,
                                             uint32_t* s_hist, uint32_t* s_wave, uint32_t* s_out,
                                             uint32_t* s_red, EMIT emit) {
    uint32_t kmax, kmin, count;
    block_key_range<R>(key, idx, s_red, kmax, kmin, count);
    if (count <= k) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (idx[r] != kNoItem) emit(key[r], idx[r]);
        return;
    }
    uint32_t need = k;                                // items still to take from the current prefix
    int hi = kmax == kmin ? -1 : 31 - __clz(kmax ^ kmin);   // highest bit in which valid keys differ
    // the key bits above `hi` of the k-th key (none when the keys differ in bit 31)
    uint32_t prefix = hi < 0 ? kmax : (hi == 31 ? 0u : kmax >> (hi + 1));
    uint32_t beyond, in_bin, total;
    while (hi >= 0) {
        const int shift = hi >= 11 ? hi - 11 : 0;
        const uint32_t bins = 1u << (hi - shift + 1);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (idx[r] != kNoItem && (key[r] >> hi >> 1) == prefix)
                atomicAdd(&s_hist[(key[r] >> shift) & (bins - 1u)], 1u);
        __syncthreads();
        const uint32_t d = find_bin<true>(s_hist, bins, need, s_wave, s_out, beyond, in_bin, total);
        need -= beyond;
        prefix = (prefix << (hi - shift + 1)) | d;
        hi = shift - 1;
        if (in_bin == need) {
            // the whole bin is taken: the k best are the keys whose prefix is at least this one
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (idx[r] != kNoItem && (key[r] >> shift) >= prefix) emit(key[r], idx[r]);
            return;
        }
    }
    const uint32_t T = prefix;                        // the k-th key; 1 <= need < its count
    // the need lowest indices among the keys equal to T (index < 2^22)
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (idx[r] != kNoItem && key[r] == T) atomicAdd(&s_hist[idx[r] >> 11], 1u);
    __syncthreads();
    const uint32_t ihi = find_bin<false>(s_hist, 2048, need, s_wave, s_out, beyond, in_bin, total);
    need -= beyond;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (idx[r] != kNoItem && key[r] == T && (idx[r] >> 11) == ihi) atomicAdd(&s_hist[idx[r] & 0x7FFu], 1u);
    __syncthreads();
    const uint32_t imax = (ihi << 11) | find_bin<false>(s_hist, 2048, need, s_wave, s_out, beyond, in_bin, total);
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (idx[r] != kNoItem && (key[r] > T || (key[r] == T && idx[r] <= imax))) emit(key[r], idx[r]);
}

// One stage: workgroup b takes items 4096 b .. 4096 b + 4095 (predictions
// when FROM_PRED, else the previous stage's keys and indices) and writes its
// k best to slots k b .. k b + k - 1 (empty slots marked kNoItem).
template <bool FROM_PRED>
__global__ __launch_bounds__(kSelThreads) void select_stage_kernel(const float* __restrict__ pred,
                                                                   const uint32_t* __restrict__ in_key,
                                                                   const uint32_t* __restrict__ in_idx,
                                                                   uint32_t count, uint32_t k,
                                                                   uint32_t* __restrict__ out_key,
                                                                   uint32_t* __restrict__ out_idx) {
    __shared__ uint32_t s_hist[4096];
    __shared__ uint32_t s_wave[kSelThreads / 64];
    __shared__ uint32_t s_red[3 * (kSelThreads / 64)];
    __shared__ uint32_t s_out[3];
    __shared__ uint32_t s_count;
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < 4096; i += kSelThreads) s_hist[i] = 0u;
    if (t == 0) s_count = 0u;
    uint32_t key[4], idx[4];
    const uint32_t i0 = blockIdx.x * kStageSlice + 4u * t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t i = i0 + r;
        if (FROM_PRED) {
            key[r] = i < count ? mono_key(pred[i]) : 0u;
            idx[r] = i < count ? i : kNoItem;
        } else {
            key[r] = i < count ? in_key[i] : 0u;
            idx[r] = i < count ? in_idx[i] : kNoItem;
        }
    }
    __syncthreads();
    uint32_t* ok = out_key + (size_t)blockIdx.x * k;
    uint32_t* oi = out_idx + (size_t)blockIdx.x * k;
    block_select<4>(key, idx, k, s_hist, s_wave, s_out, s_red, [&](uint32_t kk, uint32_t ii) {
        const uint32_t p = atomicAdd(&s_count, 1u);
        if (p < k) {
            ok[p] = kk;
            oi[p] = ii;
        }
    });
    __syncthreads();
    for (uint32_t p = s_count + t; p < k; p += kSelThreads) {
        ok[p] = 0u;
        oi[p] = kNoItem;
    }
}

// The last stage (one workgroup, count <= 1024 R): the k best become the
// candidates, with their poses when `poses` is given.
template <bool FROM_PRED, int R>
__global__ __launch_bounds__(kSelThreads) void select_final_kernel(const float* __restrict__ pred,
                                                                   const uint32_t* __restrict__ in_key,
                                                                   const uint32_t* __restrict__ in_idx,
                                                                   uint32_t count, uint32_t k,
                                                                   const float* __restrict__ poses,
                                                                   uint32_t* __restrict__ cand,
                                                                   float* __restrict__ cand_poses) {
    __shared__ uint32_t s_hist[4096];
    __shared__ uint32_t s_wave[kSelThreads / 64];
    __shared__ uint32_t s_red[3 * (kSelThreads / 64)];
    __shared__ uint32_t s_out[3];
    __shared__ uint32_t s_count;
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < 4096; i += kSelThreads) s_hist[i] = 0u;
    if (t == 0) s_count = 0u;
    uint32_t key[R], idx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * kSelThreads + t;           // coalesced
        if (FROM_PRED) {
            key[r] = i < count ? mono_key(pred[i]) : 0u;
            idx[r] = i < count ? i : kNoItem;
        } else {
            key[r] = i < count ? in_key[i] : 0u;
            idx[r] = i < count ? in_idx[i] : kNoItem;
        }
    }
    __syncthreads();
    // the chosen indices go to LDS (the histogram's space, free again once
    // the selection is made) and then out, with their poses, by all threads
    uint32_t* s_cand = s_hist;
    block_select<R>(key, idx, k, s_hist, s_wave, s_out, s_red, [&](uint32_t, uint32_t ii) {
        const uint32_t p = atomicAdd(&s_count, 1u);
        if (p < k) s_cand[p] = ii;
    });
    __syncthreads();
    const uint32_t got = min(s_count, k);
    for (uint32_t p = t; p < got; p += kSelThreads) cand[p] = s_cand[p];
    if (poses) {
        for (uint32_t j = t; j < 12u * got; j += kSelThreads) {
            const uint32_t p = j / 12u, e = j - 12u * p;
            cand_poses[j] = poses[12 * (size_t)s_cand[p] + e];
        }
    }
}

// ---------------------------------------------------------------- top-k ----
// Keys order candidates by value (descending) and index (ascending on ties):
// mono_key(value) << 32 | ~index.  NaN ranks below everything.
__device__ __forceinline__ unsigned long long rank_key(float v, uint32_t idx) {
    return ((unsigned long long)mono_key(v) << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

// Final pick among the rescored candidates, and the order of a top-k set:
// slot j holds candidate cand[j] with value vals[j] (vals[cand[j]] when
// `gather`); the k best come out best first, ties to the lower candidate
// index.  Keys are distinct (the candidate index is in the low word), so each
// slot's rank is the number of larger keys, and the k best write themselves.
__global__ __launch_bounds__(kMaxRescore) void final_select_kernel(const float* __restrict__ vals,
                                                                   const uint32_t* __restrict__ cand,
                                                                   uint32_t kr, uint32_t k, int gather,
                                                                   uint32_t* __restrict__ idx_out,
                                                                   float* __restrict__ val_out) {
    __shared__ __align__(16) unsigned long long s_key[kMaxRescore + 2];
    const uint32_t i = threadIdx.x;
    unsigned long long key = 0ull;
    float v = 0.0f;
    if (i < kr) {
        v = gather ? vals[cand[i]] : vals[i];
        key = rank_key(v, cand[i]);
        s_key[i] = key;
    }
    if (i == 0 && (kr & 1u)) s_key[kr] = 0ull;       // pads an odd count: ranks above no key
    __syncthreads();
    if (i >= kr) return;
    uint32_t rank = 0;
    const ulonglong2* kp = reinterpret_cast<const ulonglong2*>(s_key);
#pragma unroll 4
    for (uint32_t j = 0; j < (kr + 1) / 2; ++j) {
        const ulonglong2 kk = kp[j];
        rank += (kk.x > key ? 1u : 0u) + (kk.y > key ? 1u : 0u);
    }
    if (rank < k) {
        idx_out[rank] = cand[i];
        if (val_out) val_out[rank] = v;
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_patch(const DevMap& m, int f, const int i0[3], __bf16* out_bf16, float* out_f32,
                        hipStream_t s) {
    const int64_t rows = (int64_t)kPatchRun * f * f;
    const int threads = rows >= 256 ? 256 : (int)((rows + 63) / 64 * 64);
    hipLaunchKernelGGL(patch_kernel, dim3(kPatchCells / kPatchRun), dim3(threads), 0, s, m, f, i0[0], i0[1],
                       i0[2], out_bf16, out_f32);
    return hipGetLastError();
}

hipError_t launch_trunk(const TrunkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(trunk_front_kernel, dim3(kTrunkBlocks), dim3(kTrunkThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(trunk_conv3_kernel, dim3(4), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(trunk_conv4_kernel, dim3(4), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(trunk_fc1_kernel, dim3(kHidden / 16), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlp(const float* poses, uint32_t n, const float poi[3], float dist_mean,
                      float dist_scale, const float* c, const float* w1d, const __bf16* w2,
                      const float* b2, const float* w3, float b3, float out_scale, float* pred,
                      int cu_count, hipStream_t s) {
    const size_t lds = kMlpLds;
    static std::atomic<size_t> lds_set[64];
    hipError_t e = allow_dynamic_lds((const void*)mlp_kernel, lds, lds_set, 64);
    if (e != hipSuccess) return e;
    const uint32_t groups = (n + 31) / 32;
    uint32_t blocks = (groups + kMlpWaves - 1) / kMlpWaves;
    const uint32_t cap = (uint32_t)cu_count;     // one block per CU holds W2 in its LDS
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(mlp_kernel, dim3(blocks), dim3(kMlpWaves * 64), lds, s, poses, n, poi[0], poi[1], poi[2],
                       dist_mean, dist_scale, c, w1d, w2, b2, w3, b3, out_scale, pred);
    return hipGetLastError();
}

// Stage outputs of n items: k slots per 4096 items, and again until at most
// kFinalItems remain.
size_t select_scratch_items(uint32_t n, uint32_t k) {
    size_t most = 0;
    uint64_t count = n;
    while (count > kFinalItems) {
        count = (count + kStageSlice - 1) / kStageSlice * k;
        if (count > most) most = count;               // k <= 1024: each stage keeps at most a quarter
    }
    return most;
}

hipError_t launch_select(const float* pred, uint32_t n, uint32_t k, const float* poses, uint32_t* scratch,
                         size_t scratch_items, uint32_t* cand, float* cand_poses, hipStream_t s) {
    const uint32_t* in_key = nullptr;
    const uint32_t* in_idx = nullptr;
    uint32_t count = n;
    int flip = 0;
    while (count > kFinalItems) {
        const uint32_t blocks = (count + kStageSlice - 1) / kStageSlice;
        uint32_t* ok = scratch + (flip ? 2 * scratch_items : 0);
        uint32_t* oi = ok + scratch_items;
        if (!in_key)
            hipLaunchKernelGGL(select_stage_kernel<true>, dim3(blocks), dim3(kSelThreads), 0, s, pred, nullptr,
                               nullptr, count, k, ok, oi);
        else
            hipLaunchKernelGGL(select_stage_kernel<false>, dim3(blocks), dim3(kSelThreads), 0, s, nullptr, in_key,
                               in_idx, count, k, ok, oi);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in_key = ok;
        in_idx = oi;
        count = blocks * k;
        flip ^= 1;
    }
    // four items per thread when they fit, sixteen otherwise
#define NBT_FINAL(FP, RR)                                                                                \
    hipLaunchKernelGGL((select_final_kernel<FP, RR>), dim3(1), dim3(kSelThreads), 0, s, FP ? pred : nullptr, \
                       in_key, in_idx, count, k, poses, cand, cand_poses)
    if (!in_key) {
        if (count <= 4 * kSelThreads) NBT_FINAL(true, 4); else NBT_FINAL(true, 16);
    } else {
        if (count <= 4 * kSelThreads) NBT_FINAL(false, 4); else NBT_FINAL(false, 16);
    }
#undef NBT_FINAL
    return hipGetLastError();
}

hipError_t launch_final_select(const float* vals, const uint32_t* cand, uint32_t kr, uint32_t k, bool gather,
                               uint32_t* idx_out, float* val_out, hipStream_t s) {
    hipLaunchKernelGGL(final_select_kernel, dim3(1), dim3(kMaxRescore), 0, s, vals, cand, kr, k, gather ? 1 : 0,
                       idx_out, val_out);
    return hipGetLastError();
}

}  // namespace nbt

namespace nbt {

__global__ void bf16_to_f32_kernel(const __bf16* __restrict__ in, uint32_t n, float* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

hipError_t launch_bf16_to_f32(const __bf16* in, uint32_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

}  // namespace nbt
