// probe.hip -- probes for the measurement of the kernels' ceilings: what the
// cache levels and HBM deliver to the access patterns of a voxel walk, over a
// working set of a given size, and the issue rate of the BF16 MFMA forms the
// surrogate uses.
//
//   stream        every 16-byte piece of the buffer read once per pass, in
//                 coalesced order (the plain read bandwidth of the level the
//                 working set fits in);
//   gather        each lane reads 4-byte words at pseudo-random positions,
//                 one position per lane and load (one ray per lane, its
//                 voxels scattered over the map);
//   quad gather   the four lanes of each quad read the four words of one
//                 pseudo-random 16-byte piece (a 2x2 ray quad whose voxels
//                 fall in one row of a column tile, as in the walk's
//                 coalescing best case).
// Positions come from a xorshift sequence per lane (per quad), so no index
// array is read.  Each workgroup writes the xor of the words it read, so no
// load is dead.
#include "host.hpp"

namespace nbt {

constexpr int kProbeThreads = 256;

__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

__device__ __forceinline__ void probe_sink(uint32_t x, uint32_t* sink) {
    __shared__ uint32_t s[kProbeThreads / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t y = 0;
#pragma unroll
        for (int w = 0; w < kProbeThreads / 64; ++w) y ^= s[w];
        sink[blockIdx.x] = y;
    }
}

// n16 (16-byte pieces) a power of two; the passes x n16 reads are spread over
// all lanes, pass after pass, so that small buffers keep every lane busy.
__global__ __launch_bounds__(kProbeThreads) void probe_stream_kernel(const uint4* __restrict__ buf, uint32_t n16,
                                                                     uint32_t passes, uint32_t* __restrict__ sink) {
    uint32_t x = 0;
    const uint32_t stride = gridDim.x * kProbeThreads;
    const uint32_t total = passes * n16;
#pragma unroll 4
    for (uint32_t g = blockIdx.x * kProbeThreads + threadIdx.x; g < total; g += stride) {
        const uint4 v = buf[g & (n16 - 1u)];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    probe_sink(x, sink);
}

// words: a power of two; GROUP lanes share one 16-byte piece (GROUP = 1 or 4).
template <int GROUP>
__global__ __launch_bounds__(kProbeThreads) void probe_gather_kernel(const uint32_t* __restrict__ buf, uint32_t words,
                                                                     uint32_t loads, uint32_t* __restrict__ sink) {
    const uint32_t gid = blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t h = (gid / GROUP) * 2654435761u + 0x9E3779B9u;
    h = xorshift32(h ? h : 1u);
    const uint32_t mask = GROUP == 1 ? words - 1u : (words >> 2) - 1u;
    const uint32_t sub = GROUP == 1 ? 0u : (threadIdx.x & 3u);
    uint32_t x = 0;
#pragma unroll 8
    for (uint32_t i = 0; i < loads; ++i) {
        h = xorshift32(h);
        const uint32_t w = GROUP == 1 ? (h & mask) : ((h & mask) << 2) | sub;
        x ^= buf[w];
    }
    probe_sink(x, sink);
}

// ---- MFMA issue rate: independent BF16 accumulation chains in registers,
// no memory traffic in the loop.  Each block is 4 waves (one per SIMD); the
// launch gives every SIMD `waves_per_simd` of them.  Operands come from the
// thread index so that nothing folds; the sink takes the xor of the final
// accumulators' bits.
typedef __bf16 probe_bf16x8 __attribute__((ext_vector_type(8)));
typedef float probe_f32x4 __attribute__((ext_vector_type(4)));
typedef float probe_f32x16 __attribute__((ext_vector_type(16)));
constexpr int kProbeChains16 = 16, kProbeChains32 = 8;

__device__ __forceinline__ void probe_operands(probe_bf16x8& a, probe_bf16x8& b) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(1.0f + 0.001f * (float)((threadIdx.x + i) & 15));
        b[i] = (__bf16)(1.0f - 0.001f * (float)i);
    }
}

__global__ __launch_bounds__(kProbeThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void probe_mfma16_kernel(
    uint32_t iters, uint32_t* __restrict__ sink) {
    probe_bf16x8 a, b;
    probe_operands(a, b);
    probe_f32x4 acc[kProbeChains16];
#pragma unroll
    for (int c = 0; c < kProbeChains16; ++c) acc[c] = probe_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kProbeChains16; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains16; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) x ^= __float_as_uint(acc[c][r]);
    probe_sink(x, sink);
}

__global__ __launch_bounds__(kProbeThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void probe_mfma32_kernel(
    uint32_t iters, uint32_t* __restrict__ sink) {
    probe_bf16x8 a, b;
    probe_operands(a, b);
    probe_f32x16 acc[kProbeChains32];
#pragma unroll
    for (int c = 0; c < kProbeChains32; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kProbeChains32; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains32; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) x ^= __float_as_uint(acc[c][r]);
    probe_sink(x, sink);
}

}  // namespace nbt

using namespace nbt;

extern "C" {

int nbt_ig_probe_sink_words(const nbt_ig_ctx* ctx) { return ctx ? 8 * ctx->cu_count : 0; }

int nbt_ig_probe_memory(nbt_ig_ctx* ctx, int kind, const void* buf, size_t bytes, uint32_t count,
                        uint32_t* sink, void* stream) {
    if (!ctx || !buf || !sink) return fail(NBT_IG_EINVAL, "ctx, buf or sink is NULL");
    if (kind < NBT_IG_PROBE_STREAM || kind > NBT_IG_PROBE_QUAD_GATHER) return fail(NBT_IG_EINVAL, "unknown probe %d", kind);
    if (count < 1) return fail(NBT_IG_EINVAL, "count must be >= 1");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return fail(NBT_IG_EINVAL, "buf must be 16-byte aligned");
    if (kind == NBT_IG_PROBE_STREAM) {
        const size_t n16 = bytes / 16;
        if (bytes % 16 != 0 || n16 < 1 || (n16 & (n16 - 1)) != 0 || n16 > (1ull << 28) ||
            (uint64_t)n16 * count >= (1ull << 32))
            return fail(NBT_IG_EINVAL, "stream: bytes/16 must be a power of two, count * bytes/16 < 2^32");
    } else {
        const size_t words = bytes / 4;
        if (bytes % 4 != 0 || words < 4 || (words & (words - 1)) != 0 || words > (1ull << 31))
            return fail(NBT_IG_EINVAL, "gather: bytes/4 must be a power of two in [4, 2^31]");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(8 * ctx->cu_count), block(kProbeThreads);
    if (kind == NBT_IG_PROBE_STREAM)
        hipLaunchKernelGGL(probe_stream_kernel, grid, block, 0, s, static_cast<const uint4*>(buf),
                           (uint32_t)(bytes / 16), count, sink);
    else if (kind == NBT_IG_PROBE_GATHER)
        hipLaunchKernelGGL(probe_gather_kernel<1>, grid, block, 0, s, static_cast<const uint32_t*>(buf),
                           (uint32_t)(bytes / 4), count, sink);
    else
        hipLaunchKernelGGL(probe_gather_kernel<4>, grid, block, 0, s, static_cast<const uint32_t*>(buf),
                           (uint32_t)(bytes / 4), count, sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "probe kernel");
    return NBT_IG_OK;
}

int nbt_ig_probe_mfma(nbt_ig_ctx* ctx, int kind, int waves_per_simd, uint32_t iters, uint32_t* sink,
                      double* flops, void* stream) {
    if (!ctx || !sink) return fail(NBT_IG_EINVAL, "ctx or sink is NULL");
    if (kind != NBT_IG_PROBE_MFMA_16X16X32_BF16 && kind != NBT_IG_PROBE_MFMA_32X32X16_BF16)
        return fail(NBT_IG_EINVAL, "unknown MFMA probe %d", kind);
    if (waves_per_simd < 1 || waves_per_simd > 8) return fail(NBT_IG_EINVAL, "waves_per_simd must lie in [1, 8]");
    if (iters < 1) return fail(NBT_IG_EINVAL, "iters must be >= 1");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t blocks = (uint32_t)ctx->cu_count * (uint32_t)waves_per_simd;   // <= the sink's 8 per CU
    const bool big = kind == NBT_IG_PROBE_MFMA_32X32X16_BF16;
    if (big)
        hipLaunchKernelGGL(probe_mfma32_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, iters, sink);
    else
        hipLaunchKernelGGL(probe_mfma16_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, iters, sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "MFMA probe kernel");
    if (flops) {
        // 2 x M x N x K per instruction: 16,384 (16x16x32) or 32,768 (32x32x16)
        const double per = big ? 2.0 * 32 * 32 * 16 : 2.0 * 16 * 16 * 32;
        *flops = (double)blocks * (kProbeThreads / 64) * (double)iters * (big ? kProbeChains32 : kProbeChains16) * per;
    }
    return NBT_IG_OK;
}

}  // extern "C"
