// nbt_ig.hip -- host side of the C ABI: validation, device memory, launches.
#include "host.hpp"

using namespace nbt;

namespace {
thread_local std::string g_last_error = "no error";

// Reduction slots of nbt_ig_eval_viewpoints_noalloc: one file-scope array that
// every device holds in its own memory for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it only stands in for
// the symbol): the device address of each device's copy is looked up once, with
// that device current, and kept in g_scratch_dev.
constexpr uint32_t kNoAllocSlots = NBT_IG_NOALLOC_MAX_VIEWPOINTS;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) nbt::VpAccum scratch[kNoAllocSlots];
std::mutex g_scratch_mu;
nbt::VpAccum* g_scratch_dev[kNoAllocDevices] = {};

// Called from nbt_ig_ctx_create with `device` current.
int init_noalloc_scratch(int device) {
    if (device >= kNoAllocDevices) return NBT_IG_OK;       // the entry point refuses such devices
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return NBT_IG_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return nbt::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                      "address of the no-allocation scratch");
    e = nbt::launch_clear_slots(static_cast<nbt::VpAccum*>(ptr), kNoAllocSlots, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return nbt::hip_fail(e, "clearing the no-allocation scratch");
    g_scratch_dev[device] = static_cast<nbt::VpAccum*>(ptr);
    return NBT_IG_OK;
}
}  // namespace

namespace nbt {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? NBT_IG_ENOMEM : NBT_IG_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

}  // namespace nbt

namespace nbt {

int grow_buffer(void** p, size_t* cap, bool* async, size_t bytes, hipStream_t s, const char* what) {
    if (*cap >= bytes) return NBT_IG_OK;
    void* q = nullptr;
    bool as = true;
    hipError_t e = hipMallocAsync(&q, bytes, s);
    if (e == hipErrorNotSupported) {
        // no stream-ordered allocator: wait for this stream only, then allocate
        (void)hipGetLastError();
        as = false;
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipMalloc(&q, bytes);
    }
    if (e != hipSuccess) return hip_fail(e, what);
    if (*p) release_buffer(*p, *async, s);
    *p = q;
    *cap = bytes;
    *async = as;
    return NBT_IG_OK;
}

void release_buffer(void* p, bool async, hipStream_t s) {
    if (!p) return;
    if (async) {
        (void)hipFreeAsync(p, s);
    } else {
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
    }
}

int ensure_workspace(nbt_ig_ctx* ctx, size_t slots, hipStream_t s) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const size_t have = ctx->ws_bytes / sizeof(VpAccum);
    if (have >= slots) return NBT_IG_OK;
    size_t cap = have ? have : 1024;
    while (cap < slots) cap *= 2;
    if (cap >= (1ull << 32)) return fail(NBT_IG_EUNSUPPORTED, "too many perspectives for the workspace");
    void* p = ctx->ws;
    if (int rc = grow_buffer(&p, &ctx->ws_bytes, &ctx->ws_async, cap * sizeof(VpAccum), s, "workspace"))
        return rc;
    ctx->ws = static_cast<VpAccum*>(p);
    const hipError_t e = launch_clear_slots(ctx->ws, (uint32_t)cap, s);   // the kernels keep them zero
    if (e != hipSuccess) return hip_fail(e, "workspace clear");
    return NBT_IG_OK;
}

static int ensure_traj_workspace(nbt_ig_ctx* ctx, size_t T, hipStream_t s) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->boxes_bytes >= T * sizeof(TrajBox)) return NBT_IG_OK;
    size_t cap = ctx->boxes_bytes ? ctx->boxes_bytes / sizeof(TrajBox) : 1024;
    while (cap < T) cap *= 2;
    void* p = ctx->boxes;
    if (int rc = grow_buffer(&p, &ctx->boxes_bytes, &ctx->boxes_async, cap * sizeof(TrajBox), s,
                             "trajectory boxes"))
        return rc;
    ctx->boxes = static_cast<TrajBox*>(p);
    return NBT_IG_OK;
}

size_t traj_lds_bytes(const nbt_ig_ctx* ctx) {
    const int k = ctx->traj_waves == 4 ? 0 : ctx->traj_waves == 8 ? 1 : 2;
    size_t b = ctx->lds_budget ? ctx->lds_budget : ctx->traj_lds_share[k];
    if (b > ctx->lds_max) b = ctx->lds_max;
    return b < 12 ? 12 : b / 4 * 4;      // at least one word of bitset
}

int check_camera(const nbt_ig_camera* cam, CamParams* out) {
    if (!cam) return fail(NBT_IG_EINVAL, "camera is NULL");
    if (cam->width < 1 || cam->height < 1)
        return fail(NBT_IG_EINVAL, "camera grid %ux%u: both sides must be >= 1", cam->width, cam->height);
    if ((uint64_t)cam->width * cam->height > (1u << 22))
        return fail(NBT_IG_EUNSUPPORTED, "camera grid %ux%u exceeds 2^22 rays per perspective",
                    cam->width, cam->height);
    if (!finite_pos(cam->tan_half_fov_h) || !finite_pos(cam->tan_half_fov_v) || !finite_pos(cam->range))
        return fail(NBT_IG_EINVAL, "camera tangents and range must be finite and > 0");
    out->W = (int)cam->width;
    out->H = (int)cam->height;
    out->range = cam->range;
    out->dh = cam->range * cam->tan_half_fov_h;
    out->dv = cam->range * cam->tan_half_fov_v;
    return NBT_IG_OK;
}

int check_map(const nbt_ig_map* map) {
    if (!map || !map->enc || !map->ctx) return fail(NBT_IG_EINVAL, "map is NULL or destroyed");
    return NBT_IG_OK;
}

// Sets the storage order of dm (px, py, pz given) and returns its word count.
uint64_t set_layout_geometry(DevMap& dm, int layout) {
    dm.layout = layout;
    dm.tl = layout_tile_log2(layout);
    if (dm.tl == 0) {
        dm.nbx = dm.nby = 0;
        return (uint64_t)dm.px * dm.py * dm.pz;
    }
    const int T = 1 << dm.tl;
    dm.nbx = (dm.px + T - 1) >> dm.tl;
    dm.nby = (dm.py + T - 1) >> dm.tl;
    return (uint64_t)dm.nbx * dm.nby * (uint64_t)(T * T) * dm.pz;
}

}  // namespace nbt

// ---------------------------------------------------------------- API -------

// Rewrites the map's words in `layout` order (no check of who holds the map).
int relayout_map(nbt_ig_map* map, int layout, hipStream_t s) {
    if (map->dm.layout == layout) return NBT_IG_OK;
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    DevMap nd = map->dm;
    const uint64_t words = set_layout_geometry(nd, layout);
    if (words >= (1ull << 30)) return fail(NBT_IG_EUNSUPPORTED, "map too large for this layout");
    uint32_t* enc = nullptr;
    hipError_t e = hipMalloc(&enc, words * 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(map)");
    nd.enc = enc;
    nd.bytes = (uint32_t)(words * 4);
    e = launch_relayout(map->dm, enc, nd, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);     // the old words are read until here
    if (e != hipSuccess) {
        (void)hipFree(enc);
        return hip_fail(e, "relayout_kernel");
    }
    (void)hipFree(map->enc);
    map->enc = enc;
    map->enc_bytes = words * 4;
    map->dm = nd;
    return NBT_IG_OK;
}

extern "C" {

int nbt_ig_abi_version(void) { return NBT_IG_ABI_VERSION; }

const char* nbt_ig_last_error(void) { return g_last_error.c_str(); }

const char* nbt_ig_status_string(int s) {
    switch (s) {
        case NBT_IG_OK: return "ok";
        case NBT_IG_EINVAL: return "invalid argument";
        case NBT_IG_ENOMEM: return "out of memory";
        case NBT_IG_EDEVICE: return "device error";
        case NBT_IG_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

int nbt_ig_ctx_create(int device, nbt_ig_ctx** out) {
    if (!out) return fail(NBT_IG_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(NBT_IG_EINVAL, "device %d out of range (%d devices)", device, count);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(NBT_IG_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                    prop.gcnArchName);
    nbt_ig_ctx* ctx = new (std::nothrow) nbt_ig_ctx;
    if (!ctx) return fail(NBT_IG_ENOMEM, "host allocation failed");
    ctx->device = device;
    ctx->cu_count = prop.multiProcessorCount;
    {
        DeviceGuard g(device);
        size_t lds = prop.sharedMemPerBlock;
        if (lds > 160 * 1024) lds = 160 * 1024;
        const size_t fixed = traj_static_lds_bytes();
        ctx->lds_max = lds > fixed + 256 ? (lds - fixed - 256) / 256 * 256 : 0;
        ctx->lds_budget = 0;
        // The LDS a union workgroup may take without lowering the number of
        // its workgroups that registers allow on one CU.
        size_t per_cu = prop.maxSharedMemoryPerMultiProcessor;
        if (per_cu == 0 || per_cu > 160 * 1024) per_cu = 160 * 1024;
        const int waves[3] = {4, 8, 16};
        for (int k = 0; k < 3; ++k) {
            int blocks = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, traj_union_kernel_ptr(waves[k]),
                                                             waves[k] * 64, 0) != hipSuccess || blocks < 1) {
                (void)hipGetLastError();
                blocks = 32 / waves[k];
            }
            size_t share = per_cu / (size_t)blocks;
            share = share > fixed + 1024 ? (share - fixed - 512) / 1024 * 1024 : 4096;
            ctx->traj_lds_share[k] = std::min(share, ctx->lds_max);
        }
        // Workspaces sized for common calls up front (larger calls grow them,
        // stream-ordered).
        e = hipMalloc(&ctx->ws, 65536 * sizeof(VpAccum));
        if (e == hipSuccess) e = hipMemset(ctx->ws, 0, 65536 * sizeof(VpAccum));
        if (e == hipSuccess) ctx->ws_bytes = 65536 * sizeof(VpAccum);
        if (e == hipSuccess) e = hipMalloc(&ctx->boxes, 16384 * sizeof(TrajBox));
        if (e == hipSuccess) ctx->boxes_bytes = 16384 * sizeof(TrajBox);
        if (e != hipSuccess) {
            if (ctx->ws) (void)hipFree(ctx->ws);
            if (ctx->boxes) (void)hipFree(ctx->boxes);
            delete ctx;
            return hip_fail(e, "context workspace");
        }
        if (int rc = init_noalloc_scratch(device)) {
            (void)hipFree(ctx->ws);
            (void)hipFree(ctx->boxes);
            delete ctx;
            return rc;
        }
    }
    std::snprintf(ctx->arch, sizeof ctx->arch, "%s", prop.gcnArchName);
    *out = ctx;
    return NBT_IG_OK;
}

void nbt_ig_ctx_destroy(nbt_ig_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    release_buffer(ctx->ws, ctx->ws_async, nullptr);
    release_buffer(ctx->boxes, ctx->boxes_async, nullptr);
    release_buffer(ctx->topk_keep, ctx->topk_async, nullptr);
    if (ctx->ws_async || ctx->boxes_async || ctx->topk_async) (void)hipStreamSynchronize(nullptr);
    delete ctx;
}

int nbt_ig_create_map(nbt_ig_ctx* ctx, const float* prob, int nx, int ny, int nz, float voxel_size,
                      const float origin[3], const nbt_ig_classify* cls, void* stream,
                      nbt_ig_map** out) {
    if (!out) return fail(NBT_IG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (!prob || !origin) return fail(NBT_IG_EINVAL, "prob or origin is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
        return fail(NBT_IG_EINVAL, "map dims %dx%dx%d outside [1, 4096]", nx, ny, nz);
    const int layout = ctx->map_layout;
    DevMap geo{};
    geo.px = nx + 2; geo.py = ny + 2; geo.pz = nz + 2;
    const uint64_t padded = set_layout_geometry(geo, layout);
    if (padded >= (1ull << 30))
        return fail(NBT_IG_EUNSUPPORTED, "map %dx%dx%d: padded size must stay below 2^30 voxels", nx, ny, nz);
    if (!finite_pos(voxel_size)) return fail(NBT_IG_EINVAL, "voxel_size must be finite and > 0");
    if (!std::isfinite(origin[0]) || !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
        return fail(NBT_IG_EINVAL, "origin must be finite");
    nbt_ig_classify c = cls ? *cls : nbt_ig_classify{0.5f, 0.5f};
    if (!(c.free_threshold >= 0.0f && c.free_threshold <= c.occ_threshold && c.occ_threshold <= 1.0f))
        return fail(NBT_IG_EINVAL, "thresholds must satisfy 0 <= free <= occ <= 1");

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;

    nbt_ig_map* map = new (std::nothrow) nbt_ig_map;
    if (!map) return fail(NBT_IG_ENOMEM, "host allocation failed");
    map->ctx = ctx;
    map->voxel = voxel_size;
    std::memcpy(map->origin, origin, sizeof map->origin);
    map->cls = c;
    map->enc_bytes = padded * 4;
    hipError_t e = hipMalloc(&map->enc, map->enc_bytes);
    if (e != hipSuccess) {
        delete map;
        return hip_fail(e, "hipMalloc(map)");
    }
    DevMap& dm = map->dm;
    dm.enc = map->enc;
    dm.bytes = (uint32_t)map->enc_bytes;
    dm.nx = nx; dm.ny = ny; dm.nz = nz;
    dm.px = nx + 2; dm.py = ny + 2; dm.pz = nz + 2;
    dm.layout = geo.layout; dm.tl = geo.tl;
    dm.nbx = geo.nbx; dm.nby = geo.nby;
    dm.inv_s = 1.0f / voxel_size;
    dm.ox = origin[0]; dm.oy = origin[1]; dm.oz = origin[2];

    // Host or device source?  Host grids are staged through a device buffer.
    const size_t src_bytes = (size_t)nx * ny * nz * sizeof(float);
    const float* src = prob;
    float* staged = nullptr;
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, prob) == hipSuccess)
        on_device = attr.type == hipMemoryTypeDevice;
    else
        (void)hipGetLastError();
    int rc = NBT_IG_OK;
    unsigned int bad = 0;
    if (!on_device) {
        e = hipMalloc(&staged, src_bytes);
        if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(staging)"); goto done; }
        e = hipMemcpyAsync(staged, prob, src_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { rc = hip_fail(e, "hipMemcpyAsync(prob)"); goto done; }
        src = staged;
    }
    e = hipMalloc(&map->bad, sizeof(unsigned int));
    if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(flag)"); goto done; }
    e = hipMemsetAsync(map->bad, 0, sizeof(unsigned int), s);
    if (e != hipSuccess) { rc = hip_fail(e, "hipMemsetAsync(flag)"); goto done; }
    e = launch_encode_map(src, map->enc, dm, c.occ_threshold, c.free_threshold, map->bad, s);
    if (e != hipSuccess) { rc = hip_fail(e, "encode_map_kernel"); goto done; }
    e = hipMemcpyAsync(&bad, map->bad, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rc = hip_fail(e, "map encode"); goto done; }
    if (bad) rc = fail(NBT_IG_EINVAL, "occupancy probabilities must lie in [0, 1] (NaN found or out of range)");
done:
    if (staged) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(staged);
    }
    if (rc != NBT_IG_OK) {
        (void)hipFree(map->enc);
        if (map->bad) (void)hipFree(map->bad);
        delete map;
        return rc;
    }
    *out = map;
    return NBT_IG_OK;
}

void nbt_ig_destroy_map(nbt_ig_map* map) {
    if (!map) return;
    DeviceGuard g(map->ctx->device);
    if (map->enc) (void)hipFree(map->enc);
    if (map->bad) (void)hipFree(map->bad);
    map->enc = nullptr;
    delete map;
}

int nbt_ig_update_map(nbt_ig_map* map, const float* prob, void* stream) {
    if (int rc = check_map(map)) return rc;
    if (!prob) return fail(NBT_IG_EINVAL, "prob is NULL");
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    hipError_t e = launch_encode_map(prob, map->enc, map->dm, map->cls.occ_threshold,
                                     map->cls.free_threshold, map->bad, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "encode_map_kernel");
    return NBT_IG_OK;
}

int nbt_ig_map_check(nbt_ig_map* map, void* stream) {
    if (int rc = check_map(map)) return rc;
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    unsigned int bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, map->bad, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemsetAsync(map->bad, 0, sizeof bad, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "map check");
    if (bad) return fail(NBT_IG_EINVAL, "an update met probabilities outside [0, 1] or NaN");
    return NBT_IG_OK;
}

int nbt_ig_map_info(const nbt_ig_map* map, int* nx, int* ny, int* nz, float* voxel_size,
                    float origin[3], size_t* device_bytes) {
    if (int rc = check_map(map)) return rc;
    if (nx) *nx = map->dm.nx;
    if (ny) *ny = map->dm.ny;
    if (nz) *nz = map->dm.nz;
    if (voxel_size) *voxel_size = map->voxel;
    if (origin) std::memcpy(origin, map->origin, sizeof map->origin);
    if (device_bytes) *device_bytes = map->enc_bytes;
    return NBT_IG_OK;
}

static int eval_viewpoints_impl(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                uint32_t n, float* ig_out, uint64_t* steps_out, nbt_ig_ray_digest* trace,
                                void* stream, bool noalloc = false) {
    if (int rc = check_map(map)) return rc;
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    if (n == 0) return NBT_IG_OK;
    if (!poses || !ig_out) return fail(NBT_IG_EINVAL, "poses or ig_out is NULL");
    nbt_ig_ctx* ctx = map->ctx;
    const VpLaunch L = resolve_launch(c, ctx->vp_launch, n, ctx->cu_count);
    const uint64_t groups = vp_groups(c, L);
    if ((uint64_t)n * groups * (uint64_t)(L.waves * 64) >= (1ull << 32))
        return fail(NBT_IG_EUNSUPPORTED, "%u perspectives x %llu workgroups exceed the grid limit", n,
                    (unsigned long long)groups);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    VpAccum* ws = ctx->ws;
    if (noalloc) {
        if (n > kNoAllocSlots)
            return fail(NBT_IG_EUNSUPPORTED, "%u perspectives exceed the %u slots of the no-allocation variant", n,
                        kNoAllocSlots);
        if (ctx->device >= kNoAllocDevices || !g_scratch_dev[ctx->device])
            return fail(NBT_IG_EUNSUPPORTED, "device %d has no no-allocation scratch", ctx->device);
        ws = g_scratch_dev[ctx->device];
        if (groups > 1) {
            // the slots start at zero whatever an earlier call on this device left
            const hipError_t e = launch_clear_slots(ws, n, s);
            if (e != hipSuccess) return hip_fail(e, "clear_slots_kernel");
        }
    } else if (groups > 1) {
        if (int rc = ensure_workspace(ctx, n, s)) return rc;
        ws = ctx->ws;
    }
    hipError_t e = launch_eval_viewpoints(map->dm, c, poses, n, ig_out,
                                          reinterpret_cast<unsigned long long*>(steps_out), ws, L, s, trace);
    if (e != hipSuccess) return hip_fail(e, "ig_viewpoints_kernel");
    return NBT_IG_OK;
}

int nbt_ig_eval_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                           uint32_t n, float* ig_out, uint64_t* steps_out, void* stream) {
    return eval_viewpoints_impl(map, cam, poses, n, ig_out, steps_out, nullptr, stream);
}

int nbt_ig_eval_viewpoints_noalloc(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                   uint32_t n, float* ig_out, uint64_t* steps_out, void* stream) {
    return eval_viewpoints_impl(map, cam, poses, n, ig_out, steps_out, nullptr, stream, true);
}

int nbt_ig_trace_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                            uint32_t n, float* ig_out, uint64_t* steps_out, nbt_ig_ray_digest* out,
                            void* stream) {
    if (n > 0 && !out) return fail(NBT_IG_EINVAL, "out is NULL");
    return eval_viewpoints_impl(map, cam, poses, n, ig_out, steps_out, out, stream);
}

static int eval_trajectories_impl(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                  uint32_t n_traj, uint32_t poses_per_traj, float* ig_union,
                                  uint32_t* counts, uint64_t* visits, nbt_ig_ray_digest* trace,
                                  void* stream) {
    if (int rc = check_map(map)) return rc;
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    if (n_traj == 0) return NBT_IG_OK;
    if (!ig_union || !counts || (poses_per_traj > 0 && !poses))
        return fail(NBT_IG_EINVAL, "poses, ig_union or counts is NULL");
    const uint64_t tiles = (uint64_t)((c.W + 7) / 8) * ((c.H + 7) / 8) * poses_per_traj;
    if (tiles >= (1ull << 31)) return fail(NBT_IG_EUNSUPPORTED, "too many rays per trajectory");
    nbt_ig_ctx* ctx = map->ctx;
    const int waves = ctx->traj_waves;
    if ((uint64_t)n_traj * (uint64_t)(waves * 64) >= (1ull << 32))
        return fail(NBT_IG_EUNSUPPORTED, "%u trajectories exceed the grid limit", n_traj);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (int rc = ensure_traj_workspace(ctx, n_traj, s)) return rc;
    hipError_t e = launch_traj_boxes(map->dm, c, poses, n_traj, poses_per_traj, ctx->boxes, s);
    if (e != hipSuccess) return hip_fail(e, "traj_box_kernel");
    const size_t lds = traj_lds_bytes(ctx);
    const uint32_t pass_words = (uint32_t)(lds / 4 - 2);
    e = launch_traj_union(waves, map->dm, c, poses, poses_per_traj, n_traj, pass_words, ctx->boxes, ig_union,
                          counts, reinterpret_cast<unsigned long long*>(visits), trace, s);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? NBT_IG_ENOMEM : NBT_IG_EDEVICE,
                    "traj_union_kernel(%zu bytes of LDS of %zu): %s", lds, ctx->lds_max, hipGetErrorString(e));
    return NBT_IG_OK;
}

int nbt_ig_eval_trajectories(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                             uint32_t n_traj, uint32_t poses_per_traj, float* ig_union,
                             uint32_t* counts, uint64_t* visits, void* stream) {
    return eval_trajectories_impl(map, cam, poses, n_traj, poses_per_traj, ig_union, counts, visits, nullptr,
                                  stream);
}

int nbt_ig_trace_trajectories(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                              uint32_t n_traj, uint32_t poses_per_traj, float* ig_union, uint32_t* counts,
                              uint64_t* visits, nbt_ig_ray_digest* out, void* stream) {
    if (n_traj > 0 && poses_per_traj > 0 && !out) return fail(NBT_IG_EINVAL, "out is NULL");
    return eval_trajectories_impl(map, cam, poses, n_traj, poses_per_traj, ig_union, counts, visits, out,
                                  stream);
}

int nbt_ig_ctx_set_lds_budget(nbt_ig_ctx* ctx, size_t bytes) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->lds_budget = bytes > ctx->lds_max ? ctx->lds_max : bytes;
    return NBT_IG_OK;
}

int nbt_ig_ctx_set_map_layout(nbt_ig_ctx* ctx, int layout) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (!valid_layout(layout))
        return fail(NBT_IG_EINVAL, "unknown map layout %d", layout);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->map_layout = layout;
    return NBT_IG_OK;
}

int nbt_ig_ctx_get_map_layout(const nbt_ig_ctx* ctx, int* layout) {
    if (!ctx || !layout) return fail(NBT_IG_EINVAL, "ctx or output is NULL");
    *layout = ctx->map_layout;
    return NBT_IG_OK;
}

int nbt_ig_map_set_layout(nbt_ig_map* map, int layout, void* stream) {
    if (int rc = check_map(map)) return rc;
    if (!valid_layout(layout))
        return fail(NBT_IG_EINVAL, "unknown map layout %d", layout);
    {
        std::lock_guard<std::mutex> lk(map->ctx->mu);
        if (map->batch_refs > 0)
            return fail(NBT_IG_EINVAL, "the map is held by %d batch(es); destroy them before changing its layout",
                        map->batch_refs);
    }
    return relayout_map(map, layout, (hipStream_t)stream);
}

int nbt_ig_map_layout(const nbt_ig_map* map, int* layout) {
    if (int rc = check_map(map)) return rc;
    if (!layout) return fail(NBT_IG_EINVAL, "output is NULL");
    *layout = map->dm.layout;
    return NBT_IG_OK;
}

int nbt_ig_ctx_set_traj_waves(nbt_ig_ctx* ctx, int waves_per_group) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (!(waves_per_group == 4 || waves_per_group == 8 || waves_per_group == 16))
        return fail(NBT_IG_EINVAL, "trajectory waves per workgroup must be 4, 8 or 16 (got %d)", waves_per_group);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->traj_waves = waves_per_group;
    return NBT_IG_OK;
}

int nbt_ig_ctx_get_traj_waves(const nbt_ig_ctx* ctx, int* waves_per_group) {
    if (!ctx || !waves_per_group) return fail(NBT_IG_EINVAL, "ctx or output is NULL");
    *waves_per_group = ctx->traj_waves;
    return NBT_IG_OK;
}

int nbt_ig_ctx_info(const nbt_ig_ctx* ctx, int* cu_count, size_t* lds_per_group, size_t* lds_budget) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (cu_count) *cu_count = ctx->cu_count;
    if (lds_per_group) *lds_per_group = ctx->lds_max;
    if (lds_budget) *lds_budget = traj_lds_bytes(ctx);
    return NBT_IG_OK;
}

int nbt_ig_trace_rays(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                      uint32_t n, nbt_ig_ray_digest* out, void* stream) {
    if (int rc = check_map(map)) return rc;
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    if (n == 0) return NBT_IG_OK;
    if (!poses || !out) return fail(NBT_IG_EINVAL, "poses or out is NULL");
    if ((uint64_t)c.W * c.H * n / 256 + 1 >= (1ull << 31))
        return fail(NBT_IG_EUNSUPPORTED, "too many rays for one trace launch");
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    hipError_t e = launch_trace_rays(map->dm, c, poses, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trace_rays_kernel");
    return NBT_IG_OK;
}

int nbt_ig_trace_paths(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                       uint32_t n, const uint32_t* rays, uint32_t count, uint32_t max_len,
                       int32_t* lin_out, uint32_t* len_out, void* stream) {
    if (int rc = check_map(map)) return rc;
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    if (count == 0) return NBT_IG_OK;
    if (!poses || !rays || !len_out || (max_len > 0 && !lin_out))
        return fail(NBT_IG_EINVAL, "poses, rays, lin_out or len_out is NULL");
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    hipError_t e = launch_trace_paths(map->dm, c, poses, n, rays, count, max_len, lin_out, len_out,
                                      (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "trace_paths_kernel");
    return NBT_IG_OK;
}

int nbt_ig_ctx_set_launch(nbt_ig_ctx* ctx, const nbt_ig_launch* l) {
    if (!ctx || !l) return fail(NBT_IG_EINVAL, "ctx or launch is NULL");
    const int w = l->waves_per_group;
    if (!(w == 1 || w == 2 || w == 4 || w == 8))
        return fail(NBT_IG_EINVAL, "waves_per_group must be 1, 2, 4 or 8 (got %d)", w);
    if (l->tile_w_log2 < 0 || l->tile_w_log2 > 6)
        return fail(NBT_IG_EINVAL, "tile_w_log2 must be in 0..6 (got %d)", l->tile_w_log2);
    if (l->tiles_per_wave < 0 || l->tiles_per_wave > 4096)
        return fail(NBT_IG_EINVAL, "tiles_per_wave must be in 0..4096 (got %d)", l->tiles_per_wave);
    if (l->xcd_remap < 0 || l->xcd_remap > 65536)
        return fail(NBT_IG_EINVAL, "xcd_remap must be in 0..65536 (got %d)", l->xcd_remap);
    const int d = l->pipeline_depth == 0 ? 8 : l->pipeline_depth;
    if (!(d == 1 || d == 2 || d == 4 || d == 8))
        return fail(NBT_IG_EINVAL, "pipeline_depth must be 0 (default), 1, 2, 4 or 8 (got %d)", d);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->vp_launch = VpLaunch{w, l->tile_w_log2, l->tiles_per_wave, l->xcd_remap, d};
    return NBT_IG_OK;
}

int nbt_ig_ctx_get_launch(const nbt_ig_ctx* ctx, nbt_ig_launch* l) {
    if (!ctx || !l) return fail(NBT_IG_EINVAL, "ctx or launch is NULL");
    l->waves_per_group = ctx->vp_launch.waves;
    l->tile_w_log2 = ctx->vp_launch.tile_w_log2;
    l->tiles_per_wave = ctx->vp_launch.tiles_per_wave;
    l->xcd_remap = ctx->vp_launch.xcd_remap;
    l->pipeline_depth = ctx->vp_launch.depth;
    return NBT_IG_OK;
}

int nbt_ig_eval_cost(nbt_ig_ctx* ctx, const float* id_pos, const float* id_ig, uint32_t n_ids,
                     uint32_t n_persp, float p, const float* poses, uint32_t n_horizons, uint32_t steps,
                     const float poi[3], float tan_half_fov_h, float tan_half_fov_v, float w_i, float eps,
                     float* g_out, float* o_out, float* cost_out, void* stream) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (n_horizons == 0 || steps == 0) return NBT_IG_OK;
    if (n_ids == 0 || n_persp == 0) return fail(NBT_IG_EINVAL, "the ID buffer is empty");
    if (!id_pos || !id_ig || !poses || !poi || !g_out || !o_out)
        return fail(NBT_IG_EINVAL, "a required pointer is NULL");
    if (!(p >= 0.0f) || !std::isfinite(p) || !finite_pos(tan_half_fov_h) || !finite_pos(tan_half_fov_v) ||
        !std::isfinite(w_i) || !(eps >= 0.0f) || !std::isfinite(eps))
        return fail(NBT_IG_EINVAL, "need finite p >= 0, tangents > 0, w_i and eps >= 0");
    if (!std::isfinite(poi[0]) || !std::isfinite(poi[1]) || !std::isfinite(poi[2]))
        return fail(NBT_IG_EINVAL, "poi must be finite");
    if ((uint64_t)n_horizons * steps >= (1ull << 31) || (uint64_t)n_ids * n_persp >= (1ull << 31))
        return fail(NBT_IG_EUNSUPPORTED, "too many states or perspectives");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipError_t e = launch_eval_cost(id_pos, id_ig, n_ids, n_persp, p, poses, n_horizons, steps, poi,
                                    tan_half_fov_h, tan_half_fov_v, w_i, eps, g_out, o_out, cost_out,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "idw_query_kernel");
    return NBT_IG_OK;
}

int nbt_ig_camera_from_grid(double fov_h, double fov_v, double d_cam, double s_vox, double s_g,
                            nbt_ig_camera* out) {
    if (!out) return fail(NBT_IG_EINVAL, "out is NULL");
    if (!(fov_h > 0 && fov_h < M_PI && fov_v > 0 && fov_v < M_PI && d_cam > 0 && s_vox > 0 && s_g > 0) ||
        !std::isfinite(d_cam) || !std::isfinite(s_vox) || !std::isfinite(s_g))
        return fail(NBT_IG_EINVAL, "need 0 < fov < pi and finite d_cam, s_vox, s_g > 0");
    const double th = std::tan(fov_h / 2.0), tv = std::tan(fov_v / 2.0);
    const double spacing = s_g * s_vox;
    // 1e-9 absorbs the rounding of tan() at exact multiples of the spacing
    const double w = std::floor(2.0 * d_cam * th / spacing + 1e-9) + 1.0;
    const double h = std::floor(2.0 * d_cam * tv / spacing + 1e-9) + 1.0;
    if (w > 4194304.0 || h > 4194304.0 || w * h > 4194304.0)
        return fail(NBT_IG_EUNSUPPORTED, "grid %.0fx%.0f exceeds 2^22 rays", w, h);
    out->width = (uint32_t)w;
    out->height = (uint32_t)h;
    out->tan_half_fov_h = (float)th;
    out->tan_half_fov_v = (float)tv;
    out->range = (float)d_cam;
    return NBT_IG_OK;
}

}  // extern "C"
