// reduce.hpp -- fixed-order wavefront reductions (device code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbt {

// Butterfly over the 64 lanes: every lane ends with the same total, and the
// summation order is fixed, so results are bit-identical from run to run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace nbt
