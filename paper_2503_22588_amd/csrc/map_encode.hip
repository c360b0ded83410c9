// map_encode.hip -- occupancy probabilities -> device-resident encoded map.
//
// Each voxel is classified once (Occupied if P > occ, Free if P < free,
// Unknown otherwise) and stored as its Eq. 2 gain (1-P, P or 1) in float32
// bits, with the sign bit set for Occupied.  A one-voxel border of sentinel
// words surrounds the map (and fills the tile padding of the column orders).  The
// walk then needs one 4-byte gather and one signed compare per voxel: no
// probability, no threshold and no bounds test is evaluated per step.
// Streaming kernel, about 8 B per voxel.
#include "internal.hpp"

namespace nbt {

// Word of padded voxel (X, Y, Z) (border and tile padding: the sentinel).
__device__ __forceinline__ uint32_t encode_word(const float* __restrict__ prob, const DevMap& m, uint32_t X,
                                                uint32_t Y, uint32_t Z, float occ_thr, float free_thr,
                                                bool& any_bad) {
    if (X == 0 || Y == 0 || Z == 0 || X >= (uint32_t)m.px - 1 || Y >= (uint32_t)m.py - 1 ||
        Z >= (uint32_t)m.pz - 1)
        return kSentinel;
    const float p = prob[((size_t)(Z - 1) * (size_t)m.ny + (Y - 1)) * (size_t)m.nx + (X - 1)];
    if (!(p >= 0.0f && p <= 1.0f)) {          // also rejects NaN
        any_bad = true;
        return kGainOne;
    }
    if (p > occ_thr) return __float_as_uint(1.0f - p) | kOccBit;
    if (p < free_thr) return __float_as_uint(p) & ~kOccBit;    // -0.0 is stored as +0.0
    return kGainOne;
}

// Padded coordinates of stored word idx.
__device__ __forceinline__ void word_coords(const DevMap& m, uint32_t idx, uint32_t& X, uint32_t& Y, uint32_t& Z) {
    if (m.tl == 0) {
        X = idx % (uint32_t)m.px;
        const uint32_t yz = idx / (uint32_t)m.px;
        Y = yz % (uint32_t)m.py;
        Z = yz / (uint32_t)m.py;
    } else {
        const uint32_t t = (uint32_t)m.tl;
        const uint32_t r = idx >> (2u * t), l = idx & ((1u << (2u * t)) - 1u);
        Z = r % (uint32_t)m.pz;
        const uint32_t tile = r / (uint32_t)m.pz;
        X = ((tile % (uint32_t)m.nbx) << t) + (l & ((1u << t) - 1u));
        Y = ((tile / (uint32_t)m.nbx) << t) + (l >> t);
    }
}

// One thread per stored word, in storage order (coalesced writes).
__global__ __launch_bounds__(256) void encode_map_kernel(const float* __restrict__ prob,
                                                         uint32_t* __restrict__ enc, DevMap m,
                                                         float occ_thr, float free_thr,
                                                         unsigned int* __restrict__ bad) {
    const uint32_t total = m.bytes / 4u;
    const uint32_t stride = gridDim.x * blockDim.x;
    bool any_bad = false;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        uint32_t X, Y, Z;
        word_coords(m, idx, X, Y, Z);
        enc[idx] = encode_word(prob, m, X, Y, Z, occ_thr, free_thr, any_bad);
    }
    if (any_bad) atomicOr(bad, 1u);
}

// One thread per destination word: the word of the same padded voxel in the
// source order (the sentinel for the padding of whole tiles).
__global__ __launch_bounds__(256) void relayout_kernel(const uint32_t* __restrict__ src, DevMap sm,
                                                       uint32_t* __restrict__ dst, DevMap dm) {
    const uint32_t total = dm.bytes / 4u;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        uint32_t X, Y, Z;
        word_coords(dm, idx, X, Y, Z);
        uint32_t w = kSentinel;
        if (X < (uint32_t)dm.px && Y < (uint32_t)dm.py && Z < (uint32_t)dm.pz)
            w = src[voxel_offset(sm, (int)X - 1, (int)Y - 1, (int)Z - 1) / 4u];
        dst[idx] = w;
    }
}

hipError_t launch_relayout(const DevMap& src, uint32_t* dst, const DevMap& dstm, hipStream_t s) {
    const uint64_t total = dstm.bytes / 4u;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(relayout_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src.enc, src, dst, dstm);
    return hipGetLastError();
}

hipError_t launch_encode_map(const float* prob, uint32_t* enc, const DevMap& m, float occ_thr,
                             float free_thr, unsigned int* bad_flag, hipStream_t s) {
    const uint64_t total = m.bytes / 4u;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(encode_map_kernel, dim3((unsigned)blocks), dim3(256), 0, s, prob, enc, m,
                       occ_thr, free_thr, bad_flag);
    return hipGetLastError();
}

}  // namespace nbt
