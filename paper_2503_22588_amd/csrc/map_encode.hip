// map_encode.hip -- occupancy probabilities -> device-resident encoded map.
//
// Each voxel is classified once (Occupied if P > occ, Free if P < free,
// Unknown otherwise) and stored as its Eq. 2 gain (1-P, P or 1) in float32
// bits, with the sign bit set for Occupied.  A one-voxel border of sentinel
// words surrounds the map.  The walk then needs one 4-byte gather and one
// signed compare per voxel: no probability, no threshold and no bounds
// test is evaluated per step.  Streaming kernel, about 8 B per voxel.
#include "internal.hpp"

namespace nbt {

__global__ __launch_bounds__(256) void encode_map_kernel(const float* __restrict__ prob,
                                                         uint32_t* __restrict__ enc, DevMap m,
                                                         float occ_thr, float free_thr,
                                                         unsigned int* __restrict__ bad) {
    const uint32_t px = (uint32_t)m.px, py = (uint32_t)m.py, pz = (uint32_t)m.pz;
    const uint32_t total = px * py * pz;
    const uint32_t stride = gridDim.x * blockDim.x;
    bool any_bad = false;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const uint32_t x = idx % px;
        const uint32_t yz = idx / px;
        const uint32_t y = yz % py;
        const uint32_t z = yz / py;
        uint32_t word;
        if (x == 0 || y == 0 || z == 0 || x == px - 1 || y == py - 1 || z == pz - 1) {
            word = kSentinel;
        } else {
            const float p = prob[((size_t)(z - 1) * (size_t)m.ny + (y - 1)) * (size_t)m.nx + (x - 1)];
            if (!(p >= 0.0f && p <= 1.0f)) {          // also rejects NaN
                any_bad = true;
                word = kGainOne;
            } else if (p > occ_thr) {
                word = __float_as_uint(1.0f - p) | kOccBit;
            } else if (p < free_thr) {
                word = __float_as_uint(p) & ~kOccBit;  // -0.0 is stored as +0.0
            } else {
                word = kGainOne;
            }
        }
        enc[idx] = word;
    }
    if (any_bad) atomicOr(bad, 1u);
}

hipError_t launch_encode_map(const float* prob, uint32_t* enc, const DevMap& m, float occ_thr,
                             float free_thr, unsigned int* bad_flag, hipStream_t s) {
    const uint64_t total = (uint64_t)m.px * m.py * m.pz;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(encode_map_kernel, dim3((unsigned)blocks), dim3(256), 0, s, prob, enc, m,
                       occ_thr, free_thr, bad_flag);
    return hipGetLastError();
}

}  // namespace nbt
