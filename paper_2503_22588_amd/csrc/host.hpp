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

int ensure_workspace(nbt_ig_ctx* ctx, size_t slots);
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
    size_t ws_cap = 0;              // slots allocated
    nbt::VpLaunch vp_launch{4, 3, 0, 0, 8};  // 4 waves, 8x8 tiles, tiles/wave balanced per camera, no remap, 8 gathers in flight
    size_t lds_max = 0;             // device limit of LDS per workgroup (bytes)
    size_t lds_budget = 0;          // LDS a trajectory bitset may use (bytes)
    int traj_waves = 8;             // wavefronts per trajectory workgroup (4, 8, 16)
    int map_layout = NBT_IG_LAYOUT_COLUMN4;  // storage order of maps created next
    // trajectory workspace
    nbt::TrajBox* boxes = nullptr;
    uint32_t* over_list = nullptr;
    size_t traj_cap = 0;
    nbt::TrajMeta* meta = nullptr;       // device
    nbt::TrajMeta* meta_host = nullptr;  // pinned
    uint32_t* gbits = nullptr;
    size_t gbits_words = 0;
    unsigned long long* topk_keep = nullptr;   // top-k selection scratch
    size_t topk_cap = 0;
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
