// host.hpp -- host-side objects and helpers shared by the C-ABI translation units.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.hpp"

namespace nbt {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Makes the context's device current for the duration of a call and
// restores the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

// Grows *p to `bytes` (when smaller than *cap bytes) in the order of stream s:
// the new buffer is allocated and the old one released as stream-ordered
// operations, so no other stream of the process waits.  *async records which
// allocator owns *p (release_buffer needs it).
int grow_buffer(void** p, size_t* cap, bool* async, size_t bytes, hipStream_t s, const char* what);
void release_buffer(void* p, bool async, hipStream_t s);

int ensure_workspace(nbt_ig_ctx* ctx, size_t slots, hipStream_t s);
// LDS bytes of one trajectory workgroup's bitset (with its two extra words)
// for the context's current budget and workgroup size.
size_t traj_lds_bytes(const nbt_ig_ctx* ctx);
int check_camera(const nbt_ig_camera* cam, CamParams* out);
int check_map(const nbt_ig_map* map);

}  // namespace nbt

// ---- objects behind the opaque handles ----

struct nbt_ig_ctx {
    int device = 0;
    int cu_count = 0;
    char arch[64] = {0};
    std::mutex mu;
    nbt::VpAccum* ws = nullptr;          // per-perspective reduction slots, kept zeroed
    size_t ws_bytes = 0;
    bool ws_async = false;
    nbt::VpLaunch vp_launch{4, 3, 0, 0, 8};  // 4 waves, 8x8 tiles, tiles/wave balanced per camera, no remap, 8 gathers in flight
    size_t lds_max = 0;             // device limit of LDS per workgroup (bytes)
    size_t lds_budget = 0;          // LDS a trajectory bitset may use (bytes); 0 = traj_lds_share
    size_t traj_lds_share[3] = {0, 0, 0};  // LDS per workgroup that keeps the union kernel's occupancy (4/8/16 waves)
    int traj_waves = 8;             // wavefronts per trajectory workgroup (4, 8, 16)
    int map_layout = NBT_IG_LAYOUT_COLUMN4;  // storage order of maps created next
    // trajectory workspace
    nbt::TrajBox* boxes = nullptr;
    size_t boxes_bytes = 0;
    bool boxes_async = false;
    unsigned long long* topk_keep = nullptr;   // top-k selection scratch
    size_t topk_bytes = 0;
    bool topk_async = false;
};

struct nbt_ig_map {
    nbt_ig_ctx* ctx = nullptr;
    unsigned int* bad = nullptr;    // set by encodes that met an invalid probability
    nbt::DevMap dm{};
    uint32_t* enc = nullptr;
    size_t enc_bytes = 0;
    float voxel = 0.0f;
    float origin[3] = {0, 0, 0};
    nbt_ig_classify cls{0.5f, 0.5f};
    int batch_refs = 0;             // batches holding this map's descriptor (under ctx->mu)
};

// Rewrites an encoded map in another storage order (synchronises s); callers
// check that no batch still holds the map's old descriptor.
int relayout_map(nbt_ig_map* map, int layout, hipStream_t s);
