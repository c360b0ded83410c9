// surrogate.hpp -- sizes and launchers of the learned IG surrogate (library-internal).
#pragma once

#include "internal.hpp"

namespace nbt {

constexpr int kGrid = 32;                          // patch cells per axis
constexpr int kPatchCells = kGrid * kGrid * kGrid;
constexpr int kFeat = 512;                         // trunk output: 64 channels x 2^3
constexpr int kHidden = 256;                       // MLP width
constexpr int kMaxRescore = 1024;                  // most candidates kept by top-k / rescored exactly
constexpr uint32_t kMaxCandidates = 1u << 22;      // candidate index fits 22 bits (slot packing)
constexpr int kConvIn[4] = {2, 16, 32, 64};
constexpr int kConvOut[4] = {16, 32, 64, 64};

hipError_t launch_patch(const DevMap& m, int f, const int i0[3], __bf16* out_bf16, float* out_f32,
                        hipStream_t s);
hipError_t launch_conv(const __bf16* in, int cin, int s_in, const __bf16* w, const float* bias, int cout,
                       int kpad, __bf16* out, hipStream_t s);
hipError_t launch_fc1_feature(const __bf16* feat, const __bf16* w1f, const float* b1, float* c,
                              hipStream_t s);
hipError_t launch_mlp(const float* poses, uint32_t n, const float poi[3], float dist_mean,
                      float dist_scale, const float* c, const float* w1d, const __bf16* w2,
                      const float* b2, const float* w3, float b3, float out_scale, float* pred,
                      int cu_count, hipStream_t s);
// Keys the top-k scratch must hold for n values (two ping-pong halves).
size_t topk_scratch_keys(uint32_t n, uint32_t k);
hipError_t launch_topk(const float* vals, uint32_t n, uint32_t k, unsigned long long* scratch,
                       uint32_t* idx_out, hipStream_t s);
hipError_t launch_gather_poses(const float* poses, const uint32_t* idx, uint32_t k, float* out,
                               hipStream_t s);
hipError_t launch_final_select(const float* ig_exact, const uint32_t* cand, uint32_t kr, uint32_t k,
                               uint32_t* idx_out, float* ig_out, hipStream_t s);
hipError_t launch_gather_values(const float* vals, const uint32_t* idx, uint32_t k, float* out, hipStream_t s);
hipError_t launch_bf16_to_f32(const __bf16* in, uint32_t n, float* out, hipStream_t s);

}  // namespace nbt
