// surrogate.hip -- learned IG surrogate: patch, conv3d trunk and MLP on BF16
// MFMA (FP32 accumulation), top-k selection and the final pick after exact
// rescoring.
//
// Matrix fragments follow v_mfma_f32_16x16x32_bf16 (gfx950): for lane l,
// A (16 x 32) row l%16 holds k = (l/16)*8 .. +7, B (32 x 16) column l%16 holds
// the same k, and the 16 x 16 result gives lane l column l%16, rows
// (l/16)*4 .. +3.
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
// One thread per cell: occupied and unknown voxel counts over the cell's f^3
// voxels (voxels outside the map count as neither), divided by f^3.
__global__ __launch_bounds__(256) void patch_kernel(DevMap m, int f, int i0x, int i0y, int i0z,
                                                    __bf16* __restrict__ out_bf16,
                                                    float* __restrict__ out_f32) {
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= kPatchCells) return;
    const int cx = cell % kGrid, cy = (cell / kGrid) % kGrid, cz = cell / (kGrid * kGrid);
    const __amdgpu_buffer_rsrc_t rs = map_rsrc(m);
    uint32_t occ = 0, unk = 0;
    for (int dz = 0; dz < f; ++dz) {
        const int z = i0z + cz * f + dz;
        if (z < 0 || z >= m.nz) continue;
        for (int dy = 0; dy < f; ++dy) {
            const int y = i0y + cy * f + dy;
            if (y < 0 || y >= m.ny) continue;
            for (int dx = 0; dx < f; ++dx) {
                const int x = i0x + cx * f + dx;
                if (x < 0 || x >= m.nx) continue;
                const uint32_t w = load_word(rs, voxel_offset(m, x, y, z));
                occ += (w & kOccBit) ? 1u : 0u;
                unk += (w == kGainOne) ? 1u : 0u;
            }
        }
    }
    const float vol = (float)(f * f * f);
    const float fo = (float)occ / vol, fu = (float)unk / vol;
    if (out_bf16) {
        out_bf16[cell] = (__bf16)fo;
        out_bf16[kPatchCells + cell] = (__bf16)fu;
    }
    if (out_f32) {
        out_f32[cell] = fo;
        out_f32[kPatchCells + cell] = fu;
    }
}

// ---------------------------------------------------------------- conv -----
// Implicit GEMM: out[n][m] = ReLU(bias[n] + sum_k W[n][k] A[m][k]) with m an
// output position (z, y, x), k = ci*27 + (dz*3 + dy)*3 + dx and
// A[m][k] = in[ci][2z+dz-1][2y+dy-1][2x+dx-1] (zero outside).  One workgroup
// per 16 x 16 output tile; its S waves split the K = cin*27 reduction (chunk c
// of 32 goes to wave c % S), and wave 0 adds the S partial tiles in a fixed
// order, so the deep layers (few output tiles, long K) still spread over many
// waves and the result does not depend on timing.  W is bf16 [cout][kpad],
// zero padded to kpad.
template <int S>
__global__ __launch_bounds__(S * 64) void conv_kernel(const __bf16* __restrict__ in, int cin, int s_in,
                                                      const __bf16* __restrict__ w,
                                                      const float* __restrict__ bias, int cout, int kpad,
                                                      __bf16* __restrict__ out) {
    const int so = s_in / 2;
    const int M = so * so * so;
    const int ntiles = cout / 16;
    const int tile = blockIdx.x;
    const int mt = tile / ntiles, nt = tile - mt * ntiles;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    const int m = mt * 16 + row;
    const int z = m / (so * so), y = (m / so) % so, x = m % so;
    const int K = cin * 27;
    const int n = nt * 16 + row;
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = wave * 32; k0 < kpad; k0 += S * 32) {
        bf16x8_t a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kq * 8 + e;
            __bf16 v = (__bf16)0.0f;
            if (k < K && m < M) {
                const int ci = k / 27, tap = k - ci * 27;
                const int iz = 2 * z + tap / 9 - 1, iy = 2 * y + (tap / 3) % 3 - 1, ix = 2 * x + tap % 3 - 1;
                if (iz >= 0 && iz < s_in && iy >= 0 && iy < s_in && ix >= 0 && ix < s_in)
                    v = in[((size_t)ci * s_in + iz) * s_in * s_in + (size_t)iy * s_in + ix];
            }
            a[e] = v;
        }
        b = *reinterpret_cast<const bf16x8_t*>(w + (size_t)n * kpad + k0 + kq * 8);
        acc = mfma16(a, b, acc);
    }
    if constexpr (S > 1) {
        __shared__ f32x4_t part[S][64];
        part[wave][lane] = acc;
        __syncthreads();
        if (wave != 0) return;
#pragma unroll
        for (int q = 1; q < S; ++q) acc += part[q][lane];
    }
    const int ncol = nt * 16 + row;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mo = mt * 16 + kq * 4 + r;
        if (mo < M) {
            const float v = acc[r] + bias[ncol];
            out[(size_t)ncol * M + mo] = (__bf16)(v > 0.0f ? v : 0.0f);
        }
    }
}

// c[n] = b1[n] + sum_k W1f[n][k] f[k]: the pose-independent part of fc1.
// Sixteen lanes per output: lane j sums k = j, j + 16, ... (32 terms), then a
// fixed butterfly adds the sixteen partial sums.
__global__ __launch_bounds__(256) void fc1_feature_kernel(const __bf16* __restrict__ feat,
                                                          const __bf16* __restrict__ w1f,
                                                          const float* __restrict__ b1,
                                                          float* __restrict__ c) {
    const int n = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    float s = 0.0f;
    for (int k = j; k < kFeat; k += 16) s += (float)w1f[(size_t)n * kFeat + k] * (float)feat[k];
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) s += __shfl_xor(s, d, 16);
    if (j == 0) c[n] = b1[n] + s;
}

// ---------------------------------------------------------------- MLP ------
// Per pose: h1 = ReLU(c + W1d [u, dn]) (FP32, stored BF16), h2 = ReLU(W2 h1 +
// b2) on MFMA with W2 staged in LDS (rows padded to 264 halves so the 16
// lanes reading one k-slice of 16 rows hit distinct banks), y = out_scale *
// (W3 . h2 + b3).  One workgroup of 8 waves per CU shares the LDS copy of W2
// (and of c, W1d, b2, W3); each wave takes 16 poses at a time.
constexpr int kW2Stride = kHidden + 8;
constexpr int kMlpWaves = 8;
constexpr size_t kMlpLds = (size_t)kHidden * kW2Stride * sizeof(__bf16) + (size_t)kHidden * 7 * sizeof(float);

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
    float* sc = sw1d + 4 * kHidden;
    float* sb2 = sc + kHidden;
    float* sw3 = sb2 + kHidden;
    for (int i = threadIdx.x; i < kHidden * kHidden / 8; i += blockDim.x) {
        const int r = (i * 8) / kHidden, k = (i * 8) % kHidden;
        *reinterpret_cast<bf16x8_t*>(sw2 + r * kW2Stride + k) =
            *reinterpret_cast<const bf16x8_t*>(w2 + (size_t)r * kHidden + k);
    }
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        *reinterpret_cast<float4*>(sw1d + 4 * i) = *reinterpret_cast<const float4*>(w1d + 4 * i);
        sc[i] = c[i];
        sb2[i] = b2[i];
        sw3[i] = w3[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    const uint32_t ntile = (n + 15) / 16;
    const uint32_t wave_global = blockIdx.x * kMlpWaves + (threadIdx.x >> 6);
    const uint32_t waves = gridDim.x * kMlpWaves;
    for (uint32_t t = wave_global; t < ntile; t += waves) {
        const uint32_t p = t * 16 + row;
        float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f, dn = 0.0f;
        if (p < n) {
            const float vx = poses[12 * (size_t)p + 9] - px;
            const float vy = poses[12 * (size_t)p + 10] - py;
            const float vz = poses[12 * (size_t)p + 11] - pz;
            const float d = sqrtf(vx * vx + vy * vy + vz * vz);
            const float inv = d > 0.0f ? 1.0f / d : 0.0f;
            u0 = vx * inv;
            u1 = vy * inv;
            u2 = vz * inv;
            dn = (d - dist_mean) / dist_scale;
        }
        // output-stationary: the 16 column tiles of h2 stay in registers while
        // h1 is produced one 32-wide k-slice at a time
        f32x4_t acc[kHidden / 16];
#pragma unroll
        for (int nt = 0; nt < kHidden / 16; ++nt) acc[nt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
        for (int ks = 0; ks < kHidden / 32; ++ks) {
            bf16x8_t a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = ks * 32 + kq * 8 + e;
                const float4 wd = *reinterpret_cast<const float4*>(sw1d + 4 * k);
                float h = sc[k] + wd.x * u0 + wd.y * u1 + wd.z * u2 + wd.w * dn;
                a[e] = (__bf16)(h > 0.0f ? h : 0.0f);
            }
            const __bf16* bk = sw2 + row * kW2Stride + ks * 32 + kq * 8;
#pragma unroll
            for (int nt = 0; nt < kHidden / 16; ++nt)
                acc[nt] = mfma16(a, *reinterpret_cast<const bf16x8_t*>(bk + nt * 16 * kW2Stride), acc[nt]);
        }
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int nt = 0; nt < kHidden / 16; ++nt) {
            const int col = nt * 16 + row;
            const float bb = sb2[col], ww = sw3[col];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h2 = acc[nt][r] + bb;
                part[r] += ww * (h2 > 0.0f ? h2 : 0.0f);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) part[r] += __shfl_xor(part[r], o, 64);
        }
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t q = t * 16 + kq * 4 + r;
                if (q < n) pred[q] = out_scale * (part[r] + b3);
            }
        }
    }
}

// ---------------------------------------------------------------- top-k ----
// Keys order candidates by value (descending) and index (ascending on ties):
// (monotone bits of the value) << 32 | ~index.  NaN ranks below everything.
__device__ __forceinline__ unsigned long long rank_key(float v, uint32_t idx) {
    uint32_t b = __float_as_uint(v);
    b = (v != v) ? 0u : ((b & 0x80000000u) ? ~b : (b | 0x80000000u));
    return ((unsigned long long)b << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

// Bitonic sort, descending, of N = 1024 R keys held by a 1024-thread block,
// thread t holding keys t R .. t R + R - 1 (index i = t R + r).  A compare-
// exchange whose partner i ^ stride lies in the same thread runs on registers,
// one in the same wave on lane shuffles, and only strides of 64 R and more go
// through LDS (lds: N keys), so a 4096-key sort takes 10 barrier stages
// instead of 78.  Same network, same result as the all-LDS formulation.
template <int R>
__device__ __forceinline__ void cmpx_reg(unsigned long long (&key)[R], int t, int size, int stride) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int r2 = r ^ stride;
        if (r2 > r) {
            const int i = t * R + r;
            const bool desc = (i & size) == 0;
            const unsigned long long a = key[r], b = key[r2];
            if ((a < b) == desc) {
                key[r] = b;
                key[r2] = a;
            }
        }
    }
}

// Lane partner t ^ m: quad permutations (DPP, on the vector ALU) for m = 1, 2,
// a cross-lane permute otherwise.
__device__ __forceinline__ unsigned long long lane_xor(unsigned long long v, int m) {
    if (m == 1 || m == 2) {                           // quad_perm [1,0,3,2] / [2,3,0,1]
        const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
        const int plo = m == 1 ? __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false)
                               : __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
        const int phi = m == 1 ? __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false)
                               : __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
        return ((unsigned long long)(uint32_t)phi << 32) | (uint32_t)plo;
    }
    return __shfl_xor(v, m);
}

template <int R>
__device__ __forceinline__ void cmpx_lane(unsigned long long (&key)[R], int t, int size, int stride) {
    const int lane_mask = stride / R;                 // partner thread t ^ lane_mask, same wave
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t * R + r;
        const unsigned long long a = key[r];
        const unsigned long long b = lane_xor(a, lane_mask);
        const bool lower = (i & stride) == 0, desc = (i & size) == 0;
        const bool keep_max = lower == desc;
        key[r] = keep_max ? (a > b ? a : b) : (a < b ? a : b);
    }
}

template <int R>
__device__ void sort_desc_block(unsigned long long (&key)[R], unsigned long long* lds) {
    constexpr int N = 1024 * R;
    const int t = threadIdx.x;
    for (int size = 2; size <= N; size <<= 1) {
        int stride = size >> 1;
        if (stride >= 64 * R) {
            __syncthreads();                            // previous readers of lds are done
#pragma unroll
            for (int r = 0; r < R; ++r) lds[t * R + r] = key[r];
            for (; stride >= 64 * R; stride >>= 1) {
                __syncthreads();
                for (int p = t; p < N / 2; p += 1024) {
                    const int lo = 2 * p - (p & (stride - 1));
                    const int hi = lo + stride;
                    const bool desc = (lo & size) == 0;
                    const unsigned long long a = lds[lo], b = lds[hi];
                    if ((a < b) == desc) {
                        lds[lo] = b;
                        lds[hi] = a;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) key[r] = lds[t * R + r];
        }
        for (; stride >= R; stride >>= 1) cmpx_lane<R>(key, t, size, stride);
        for (; stride > 0; stride >>= 1) cmpx_reg<R>(key, t, size, stride);
    }
}

// Reduction pass: each block ranks 1024 R keys (from values on the first
// pass, from kept keys afterwards) and keeps its best `keep` (<= 256 R).
template <bool FROM_VALUES, int R>
__global__ __launch_bounds__(1024) void topk_pass_kernel(const float* __restrict__ vals,
                                                         const unsigned long long* __restrict__ keys_in,
                                                         uint32_t n, uint32_t keep,
                                                         unsigned long long* __restrict__ keys_out) {
    __shared__ unsigned long long s[1024 * R];
    const uint32_t base = blockIdx.x * (1024u * R);
    unsigned long long key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t g = base + threadIdx.x * R + r;
        if constexpr (FROM_VALUES)
            key[r] = g < n ? rank_key(vals[g], g) : 0ull;
        else
            key[r] = g < n ? keys_in[g] : 0ull;
    }
    sort_desc_block<R>(key, s);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x * R + r;
        if (i < keep) keys_out[(size_t)blockIdx.x * keep + i] = key[r];
    }
}

// Final pass: one block ranks all remaining keys (count <= 1024 R); writes the
// k best indices.
template <int R>
__global__ __launch_bounds__(1024) void topk_final_kernel(const float* __restrict__ vals,
                                                          const unsigned long long* __restrict__ keys,
                                                          uint32_t count, uint32_t k,
                                                          uint32_t* __restrict__ idx_out) {
    extern __shared__ unsigned long long s2[];
    unsigned long long key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x * R + r;
        if (vals)
            key[r] = i < count ? rank_key(vals[i], i) : 0ull;
        else
            key[r] = i < count ? keys[i] : 0ull;
    }
    sort_desc_block<R>(key, s2);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x * R + r;
        if (i < k) idx_out[i] = 0xFFFFFFFFu - (uint32_t)(key[r] & 0xFFFFFFFFull);
    }
}

__global__ void gather_poses_kernel(const float* __restrict__ poses, const uint32_t* __restrict__ idx,
                                    uint32_t k, float* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k * 12) out[i] = poses[12 * (size_t)idx[i / 12] + i % 12];
}

// Final pick among the rescored candidates: best exact IG first, ties to the
// lower candidate index.  Slot j holds candidate cand[j] with IG ig_exact[j];
// the key carries the slot so the IG is read back without a search.
__global__ __launch_bounds__(1024) void final_select_kernel(const float* __restrict__ ig_exact,
                                                            const uint32_t* __restrict__ cand,
                                                            uint32_t kr, uint32_t k,
                                                            uint32_t* __restrict__ idx_out,
                                                            float* __restrict__ ig_out) {
    __shared__ unsigned long long s[kMaxRescore];
    const uint32_t i = threadIdx.x;
    // low word: candidate index (< 2^22) above the slot (< 2^10), complemented
    unsigned long long key[1];
    key[0] = i < kr ? ((rank_key(ig_exact[i], 0u) & 0xFFFFFFFF00000000ull) |
                       (unsigned long long)(0xFFFFFFFFu - ((cand[i] << 10) | i)))
                    : 0ull;
    sort_desc_block<1>(key, s);
    if (i < k) {
        const uint32_t low = 0xFFFFFFFFu - (uint32_t)(key[0] & 0xFFFFFFFFull);
        const uint32_t slot = low & 1023u;
        idx_out[i] = cand[slot];
        ig_out[i] = ig_exact[slot];
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_patch(const DevMap& m, int f, const int i0[3], __bf16* out_bf16, float* out_f32,
                        hipStream_t s) {
    hipLaunchKernelGGL(patch_kernel, dim3(kPatchCells / 256), dim3(256), 0, s, m, f, i0[0], i0[1], i0[2],
                       out_bf16, out_f32);
    return hipGetLastError();
}

hipError_t launch_conv(const __bf16* in, int cin, int s_in, const __bf16* w, const float* bias, int cout,
                       int kpad, __bf16* out, hipStream_t s) {
    const int so = s_in / 2, M = so * so * so;
    const int tiles = ((M + 15) / 16) * (cout / 16);
    const int chunks = kpad / 32;
    // waves per tile: about two K chunks each, at most 16
    if (chunks >= 32)
        hipLaunchKernelGGL(conv_kernel<16>, dim3(tiles), dim3(16 * 64), 0, s, in, cin, s_in, w, bias, cout, kpad, out);
    else if (chunks >= 16)
        hipLaunchKernelGGL(conv_kernel<8>, dim3(tiles), dim3(8 * 64), 0, s, in, cin, s_in, w, bias, cout, kpad, out);
    else if (chunks >= 8)
        hipLaunchKernelGGL(conv_kernel<4>, dim3(tiles), dim3(4 * 64), 0, s, in, cin, s_in, w, bias, cout, kpad, out);
    else if (chunks >= 4)
        hipLaunchKernelGGL(conv_kernel<2>, dim3(tiles), dim3(2 * 64), 0, s, in, cin, s_in, w, bias, cout, kpad, out);
    else
        hipLaunchKernelGGL(conv_kernel<1>, dim3(tiles), dim3(64), 0, s, in, cin, s_in, w, bias, cout, kpad, out);
    return hipGetLastError();
}

hipError_t launch_fc1_feature(const __bf16* feat, const __bf16* w1f, const float* b1, float* c,
                              hipStream_t s) {
    hipLaunchKernelGGL(fc1_feature_kernel, dim3(kHidden / 16), dim3(256), 0, s, feat, w1f, b1, c);
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
    const uint32_t tiles = (n + 15) / 16;
    uint32_t blocks = (tiles + kMlpWaves - 1) / kMlpWaves;
    const uint32_t cap = (uint32_t)cu_count;     // one block per CU holds W2 in its LDS
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(mlp_kernel, dim3(blocks), dim3(kMlpWaves * 64), lds, s, poses, n, poi[0], poi[1], poi[2],
                       dist_mean, dist_scale, c, w1d, w2, b2, w3, b3, out_scale, pred);
    return hipGetLastError();
}

static uint32_t keep_for(uint32_t k) {
    uint32_t keep = 1;
    while (keep < k) keep <<= 1;
    return keep;
}

// Keys per pass block: 1024 R with R the smallest of 1, 2, 4 that keeps at
// most a quarter of them (keep <= 1024), so every pass cuts the count by 4 or
// more; short blocks sort fast, and there are many of them.
static int pass_r(uint32_t keep) { return keep <= 256 ? 1 : (keep <= 512 ? 2 : 4); }

size_t topk_scratch_keys(uint32_t n, uint32_t k) {
    const uint32_t keep = keep_for(k);
    const uint32_t chunk = 1024u * (uint32_t)pass_r(keep);
    const size_t first = (size_t)((n + chunk - 1) / chunk) * keep;
    return 2 * first + 1;
}

hipError_t launch_topk(const float* vals, uint32_t n, uint32_t k, unsigned long long* scratch,
                       uint32_t* idx_out, hipStream_t s) {
    const uint32_t keep = keep_for(k);
    const int R = pass_r(keep);
    const uint32_t chunk = 1024u * (uint32_t)R;
    const unsigned long long* keys = nullptr;
    uint32_t count = n;
    const size_t half = (size_t)((n + chunk - 1) / chunk) * keep;
    int flip = 0;
    hipError_t e = hipSuccess;
    while (count > chunk) {
        const uint32_t blocks = (count + chunk - 1) / chunk;
        unsigned long long* out = scratch + (flip ? half : 0);
#define NBT_PASS(FV, RR)                                                                           \
    hipLaunchKernelGGL((topk_pass_kernel<FV, RR>), dim3(blocks), dim3(1024), 0, s, FV ? vals : nullptr, \
                       FV ? nullptr : keys, count, keep, out)
        if (!keys) {
            if (R == 1) NBT_PASS(true, 1); else if (R == 2) NBT_PASS(true, 2); else NBT_PASS(true, 4);
        } else {
            if (R == 1) NBT_PASS(false, 1); else if (R == 2) NBT_PASS(false, 2); else NBT_PASS(false, 4);
        }
#undef NBT_PASS
        if ((e = hipGetLastError()) != hipSuccess) return e;
        keys = out;
        count = blocks * keep;
        flip ^= 1;
    }
    // one block: 1024 R keys, R = 1, 2 or 4 (count <= chunk)
    auto final = [&](auto kernel, int RF) -> hipError_t {
        const size_t lds = (size_t)1024 * RF * sizeof(unsigned long long);     // <= 32 KiB
        hipLaunchKernelGGL(kernel, dim3(1), dim3(1024), lds, s, keys ? nullptr : vals, keys, count, k, idx_out);
        return hipGetLastError();
    };
    if (count <= 1024) return final(topk_final_kernel<1>, 1);
    if (count <= 2048) return final(topk_final_kernel<2>, 2);
    return final(topk_final_kernel<4>, 4);
}

hipError_t launch_gather_poses(const float* poses, const uint32_t* idx, uint32_t k, float* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(gather_poses_kernel, dim3((k * 12 + 255) / 256), dim3(256), 0, s, poses, idx, k, out);
    return hipGetLastError();
}

hipError_t launch_final_select(const float* ig_exact, const uint32_t* cand, uint32_t kr, uint32_t k,
                               uint32_t* idx_out, float* ig_out, hipStream_t s) {
    hipLaunchKernelGGL(final_select_kernel, dim3(1), dim3(1024), 0, s, ig_exact, cand, kr, k, idx_out, ig_out);
    return hipGetLastError();
}

}  // namespace nbt

namespace nbt {

__global__ void bf16_to_f32_kernel(const __bf16* __restrict__ in, uint32_t n, float* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void gather_values_kernel(const float* __restrict__ vals, const uint32_t* __restrict__ idx,
                                     uint32_t k, float* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) out[i] = vals[idx[i]];
}

hipError_t launch_gather_values(const float* vals, const uint32_t* idx, uint32_t k, float* out, hipStream_t s) {
    hipLaunchKernelGGL(gather_values_kernel, dim3((k + 255) / 256), dim3(256), 0, s, vals, idx, k, out);
    return hipGetLastError();
}

hipError_t launch_bf16_to_f32(const __bf16* in, uint32_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

}  // namespace nbt
