// surrogate.hpp -- sizes and launchers of the learned IG surrogate (library-internal).
#pragma once

#include "internal.hpp"

namespace nbt {

constexpr int kGrid = 32;                          // patch cells per axis
constexpr int kPatchCells = kGrid * kGrid * kGrid;
constexpr int kFeat = 512;                         // trunk output: 64 channels x 2^3
constexpr int kHidden = 256;                       // MLP width
constexpr int kMaxRescore = 1024;                  // most candidates kept by a selection / rescored exactly
constexpr uint32_t kMaxCandidates = 1u << 22;      // candidate index fits 22 bits
constexpr int kConvIn[4] = {2, 16, 32, 64};
constexpr int kConvOut[4] = {16, 32, 64, 64};
constexpr int kTrunkBlocks = 64;                   // conv2's 8^3 outputs in 2^3 blocks
// Cells at most this many voxels wide are counted by the trunk's first
// launch itself; wider ones by launch_patch over the whole chip first.
constexpr int kFrontCountMaxF = 2;

// Padded reduction length of conv layer l in the library's weight order:
// conv1 k = ci*27 + tap, the others k = tap*cin + ci (tap = (dz*3+dy)*3+dx).
constexpr int conv_kpad(int l) { return (kConvIn[l] * 27 + 31) / 32 * 32; }

// Everything the one-launch trunk reads and writes.
struct TrunkArgs {
    DevMap m;
    int f;                       // map voxels per patch cell and axis
    int i0x, i0y, i0z;           // voxel of the patch's first cell corner
    const __bf16* patch;         // the counted patch [2][32^3] (cells wider than kFrontCountMaxF), or null
    const __bf16* w[4];          // conv weights [cout][conv_kpad(l)]
    const float* b[4];           // conv biases [cout]
    const __bf16* w1f;           // fc1 weights on the features [256][512]
    const float* fb1;            // fc1 bias [256]
    __bf16* act2;                // conv2 output [8][8][8][32 channels]
    __bf16* act3;                // conv3 output [4][4][4][64 channels]
    __bf16* feat;                // trunk features [512] (c*8 + z*4 + y*2 + x)
    float* c;                    // fc1's pose-independent part [256]
};

hipError_t launch_patch(const DevMap& m, int f, const int i0[3], __bf16* out_bf16, float* out_f32,
                        hipStream_t s);
hipError_t launch_trunk(const TrunkArgs& a, hipStream_t s);
hipError_t launch_mlp(const float* poses, uint32_t n, const float poi[3], float dist_mean,
                      float dist_scale, const float* c, const float* w1d, const __bf16* w2,
                      const float* b2, const float* w3, float b3, float out_scale, float* pred,
                      int cu_count, hipStream_t s);
// Items one stage buffer of launch_select holds for n predictions (0: one
// workgroup takes them all); its scratch is 4 x that many uint32.
size_t select_scratch_items(uint32_t n, uint32_t k);
// The k best predictions (ties to the lower index) as a set, with their poses.
hipError_t launch_select(const float* pred, uint32_t n, uint32_t k, const float* poses, uint32_t* scratch,
                         size_t scratch_items, uint32_t* cand, float* cand_poses, hipStream_t s);
// The k best of kr slots (slot j: candidate cand[j], value vals[j], or
// vals[cand[j]] when gather), best first, ties to the lower candidate index;
// val_out may be NULL.  kr <= kMaxRescore.
hipError_t launch_final_select(const float* vals, const uint32_t* cand, uint32_t kr, uint32_t k, bool gather,
                               uint32_t* idx_out, float* val_out, hipStream_t s);
hipError_t launch_bf16_to_f32(const __bf16* in, uint32_t n, float* out, hipStream_t s);

}  // namespace nbt
