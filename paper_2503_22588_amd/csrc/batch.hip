// batch.hip -- host side of the batched launch and of the launch-shape autotuner.
#include <vector>

#include "host.hpp"

using namespace nbt;

struct nbt_ig_batch {
    nbt_ig_ctx* ctx = nullptr;
    uint32_t n_maps = 0;
    std::vector<nbt_ig_map*> maps;      // descriptors copied below; their layout is pinned
    DevMap* d_maps = nullptr;           // descriptor table (device)
    CamParams cam{};
    uint32_t capacity = 0;              // max perspectives per run
    VpLaunch launch{};
    unsigned int* queue = nullptr;      // work-queue head (device)
    VpAccum* ws = nullptr;              // per-perspective reduction slots, kept zeroed
    uint32_t grid = 0;                  // persistent workgroups
    // the captured launch and the arguments it was built for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

void drop_graph(nbt_ig_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (auto& k : b->key) k = nullptr;
}

int set_batch_launch(nbt_ig_batch* b, const VpLaunch& L) {
    const void* k = batch_kernel_ptr(L.waves, L.depth, true);
    if (!k) return fail(NBT_IG_EINVAL, "unsupported batch launch shape");
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, L.waves * 64, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    b->launch = resolve_launch(b->cam, L);
    b->grid = (uint32_t)(per_cu * b->ctx->cu_count);
    drop_graph(b);
    return NBT_IG_OK;
}

int build_graph(nbt_ig_batch* b, const uint32_t* offsets, const float* poses, float* ig_out,
                unsigned long long* steps_out) {
    drop_graph(b);
    const VpLaunch& L = b->launch;
    const int tw = 1 << L.tile_w_log2, th = 64 >> L.tile_w_log2;
    uint32_t tiles_x = (uint32_t)((b->cam.W + tw - 1) / tw);
    uint32_t tiles = tiles_x * (uint32_t)((b->cam.H + th - 1) / th);
    uint32_t groups = vp_groups(b->cam, L);
    int tw_log2 = L.tile_w_log2, tpw = L.tiles_per_wave;
    const DevMap* maps = b->d_maps;
    uint32_t n_maps = b->n_maps, cap = b->capacity;
    CamParams cam = b->cam;
    unsigned int* queue = b->queue;
    VpAccum* ws = b->ws;

    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");

    hipKernelNodeParams reset{};
    void* reset_args[] = {&queue};
    reset.func = const_cast<void*>(batch_reset_ptr());
    reset.gridDim = dim3(1);
    reset.blockDim = dim3(1);
    reset.sharedMemBytes = 0;
    reset.kernelParams = reset_args;
    reset.extra = nullptr;
    hipGraphNode_t n_reset, n_run;
    e = hipGraphAddKernelNode(&n_reset, b->graph, nullptr, 0, &reset);
    if (e != hipSuccess) { drop_graph(b); return hip_fail(e, "hipGraphAddKernelNode(reset)"); }

    void* args[] = {&maps, &n_maps, &offsets, &cap, &cam, &poses, &groups, &tiles_x, &tiles,
                    &tw_log2, &tpw, &queue, &ig_out, &steps_out, &ws};
    hipKernelNodeParams run{};
    run.func = const_cast<void*>(batch_kernel_ptr(L.waves, L.depth, steps_out != nullptr));
    run.gridDim = dim3(b->grid);
    run.blockDim = dim3(L.waves * 64);
    run.sharedMemBytes = 0;
    run.kernelParams = args;
    run.extra = nullptr;
    e = hipGraphAddKernelNode(&n_run, b->graph, &n_reset, 1, &run);
    if (e != hipSuccess) { drop_graph(b); return hip_fail(e, "hipGraphAddKernelNode(batch)"); }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(b); return hip_fail(e, "hipGraphInstantiate"); }
    b->key[0] = offsets;
    b->key[1] = poses;
    b->key[2] = ig_out;
    b->key[3] = steps_out;
    return NBT_IG_OK;
}

bool valid_shape(const nbt_ig_launch* l) {
    const int w = l->waves_per_group, d = l->pipeline_depth == 0 ? 4 : l->pipeline_depth;
    return (w == 1 || w == 2 || w == 4 || w == 8) && l->tile_w_log2 >= 0 && l->tile_w_log2 <= 6 &&
           l->tiles_per_wave >= 0 && l->tiles_per_wave <= 4096 && l->xcd_remap >= 0 &&
           l->xcd_remap <= 65536 && (d == 1 || d == 2 || d == 4 || d == 8);
}

VpLaunch to_vp(const nbt_ig_launch& l) {
    return VpLaunch{l.waves_per_group, l.tile_w_log2, l.tiles_per_wave, l.xcd_remap,
                    l.pipeline_depth == 0 ? 4 : l.pipeline_depth};
}

nbt_ig_launch from_vp(const VpLaunch& v) {
    return nbt_ig_launch{v.waves, v.tile_w_log2, v.tiles_per_wave, v.xcd_remap, v.depth};
}

// The storage orders a layout autotuner tries (NBT_IG_LAYOUT_* are 0..3).
constexpr int kLayouts = NBT_IG_LAYOUT_COLUMN8 + 1;

int fastest_layout(const float* ms) {
    int best = 0;
    for (int l = 1; l < kLayouts; ++l)
        if (ms[l] < ms[best]) best = l;
    return best;
}

// Exhaustive search over the launch grid (4 x 3 x 4 x 3 = 144 shapes): every
// shape is applied, run once untimed (warm-up, graph rebuild) and timed over
// `reps` runs; the fastest is kept.  A search one parameter at a time was
// seen to stop in a local optimum 10 % slower than the grid's best.  Single
// waves and 2 tiles per wave are in the grid because the cross-workgroup
// combine costs a workgroup only its atomics: many small workgroups balance
// best on the large table-top workload.
template <class Apply, class Run>
int launch_search(VpLaunch start, hipStream_t s, int reps, Apply&& apply, Run&& run, VpLaunch* best_out,
                  float* best_ms_out) {
    static const int waves[] = {1, 2, 4, 8};
    static const int tiles[] = {2, 3, 4};
    static const int tpws[] = {0, 2, 4, 16};       // 0: balanced for the camera
    static const int depths[] = {2, 4, 8};
    constexpr int kW = 4, kT = 3, kP = 4, kD = 3;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    }
    auto time = [&](const VpLaunch& L, float* ms) -> int {
        if (int rc = apply(L)) return rc;
        if (int rc = run()) return rc;                 // warm-up (and graph build)
        hipError_t e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            if (int rc = run()) return rc;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        if (e != hipSuccess) return hip_fail(e, "autotune timing");
        *ms /= (float)reps;
        return NBT_IG_OK;
    };
    VpLaunch best = start;
    float best_ms = 0.0f;
    int rc = NBT_IG_OK;
    for (int a = 0; a < kW * kT * kP * kD && rc == NBT_IG_OK; ++a) {
        VpLaunch L = start;
        L.waves = waves[a % kW];
        L.tile_w_log2 = tiles[(a / kW) % kT];
        L.tiles_per_wave = tpws[(a / (kW * kT)) % kP];
        L.depth = depths[a / (kW * kT * kP)];
        float ms = 0.0f;
        rc = time(L, &ms);
        if (rc == NBT_IG_OK && (a == 0 || ms < best_ms)) {
            best_ms = ms;
            best = L;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NBT_IG_OK) return rc;
    if (int r2 = apply(best)) return r2;
    *best_out = best;
    *best_ms_out = best_ms;
    return NBT_IG_OK;
}

}  // namespace

extern "C" {

int nbt_ig_batch_create(nbt_ig_ctx* ctx, const nbt_ig_map* const* maps, uint32_t n_maps,
                        const nbt_ig_camera* cam, uint32_t max_total_viewpoints, nbt_ig_batch** out) {
    if (!out) return fail(NBT_IG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !maps || n_maps == 0) return fail(NBT_IG_EINVAL, "ctx or maps missing");
    if (max_total_viewpoints == 0) return fail(NBT_IG_EINVAL, "max_total_viewpoints must be > 0");
    CamParams c;
    if (int rc = check_camera(cam, &c)) return rc;
    std::vector<DevMap> table(n_maps);
    for (uint32_t k = 0; k < n_maps; ++k) {
        if (int rc = check_map(maps[k])) return rc;
        if (maps[k]->ctx != ctx) return fail(NBT_IG_EINVAL, "map %u belongs to another context", k);
        table[k] = maps[k]->dm;
    }
    const uint64_t groups = vp_groups(c, ctx->vp_launch);
    if ((uint64_t)max_total_viewpoints * groups >= (1ull << 32))
        return fail(NBT_IG_EUNSUPPORTED, "too many perspectives for one batch");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    nbt_ig_batch* b = new (std::nothrow) nbt_ig_batch;
    if (!b) return fail(NBT_IG_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    b->n_maps = n_maps;
    b->cam = c;
    b->capacity = max_total_viewpoints;
    hipError_t e = hipMalloc(&b->d_maps, n_maps * sizeof(DevMap));
    if (e == hipSuccess) e = hipMemcpy(b->d_maps, table.data(), n_maps * sizeof(DevMap), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->queue, 256);
    if (e == hipSuccess) e = hipMemset(b->queue, 0, 256);
    if (e == hipSuccess) e = hipMalloc(&b->ws, (size_t)max_total_viewpoints * sizeof(VpAccum));
    if (e == hipSuccess) e = hipMemset(b->ws, 0, (size_t)max_total_viewpoints * sizeof(VpAccum));
    int rc = e == hipSuccess ? set_batch_launch(b, ctx->vp_launch) : hip_fail(e, "batch allocation");
    if (rc != NBT_IG_OK) {
        nbt_ig_batch_destroy(b);
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (uint32_t k = 0; k < n_maps; ++k) {
            nbt_ig_map* mk = const_cast<nbt_ig_map*>(maps[k]);
            ++mk->batch_refs;
            b->maps.push_back(mk);
        }
    }
    *out = b;
    return NBT_IG_OK;
}

void nbt_ig_batch_destroy(nbt_ig_batch* b) {
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->ctx->mu);
        for (nbt_ig_map* mk : b->maps) --mk->batch_refs;
    }
    DeviceGuard g(b->ctx->device);
    drop_graph(b);
    if (b->d_maps) (void)hipFree(b->d_maps);
    if (b->queue) (void)hipFree(b->queue);
    if (b->ws) (void)hipFree(b->ws);
    delete b;
}

int nbt_ig_batch_run(nbt_ig_batch* b, const uint32_t* vp_offsets, const float* poses, float* ig_out,
                     uint64_t* steps_out, void* stream) {
    if (!b) return fail(NBT_IG_EINVAL, "batch is NULL");
    if (!vp_offsets || !poses || !ig_out) return fail(NBT_IG_EINVAL, "offsets, poses or ig_out is NULL");
    DeviceGuard g(b->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", b->ctx->device);
    unsigned long long* st = reinterpret_cast<unsigned long long*>(steps_out);
    if (!b->exec || b->key[0] != vp_offsets || b->key[1] != poses || b->key[2] != ig_out || b->key[3] != st)
        if (int rc = build_graph(b, vp_offsets, poses, ig_out, st)) return rc;
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch(batch)");
    return NBT_IG_OK;
}

int nbt_ig_batch_set_launch(nbt_ig_batch* b, const nbt_ig_launch* l) {
    if (!b || !l) return fail(NBT_IG_EINVAL, "batch or launch is NULL");
    if (!valid_shape(l)) return fail(NBT_IG_EINVAL, "unsupported launch shape");
    const VpLaunch L = to_vp(*l);
    if ((uint64_t)b->capacity * vp_groups(b->cam, L) >= (1ull << 32))
        return fail(NBT_IG_EUNSUPPORTED, "too many work items for this shape");
    DeviceGuard g(b->ctx->device);
    return set_batch_launch(b, L);
}

int nbt_ig_batch_get_launch(const nbt_ig_batch* b, nbt_ig_launch* l, uint32_t* persistent_groups) {
    if (!b || !l) return fail(NBT_IG_EINVAL, "batch or launch is NULL");
    *l = from_vp(b->launch);
    if (persistent_groups) *persistent_groups = b->grid;
    return NBT_IG_OK;
}

int nbt_ig_autotune_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                               uint32_t n, float* ig_out, uint64_t* steps_out, void* stream,
                               nbt_ig_launch* best, float* best_ms) {
    if (int rc = check_map(map)) return rc;
    if (!best || !best_ms) return fail(NBT_IG_EINVAL, "best or best_ms is NULL");
    if (n == 0) return fail(NBT_IG_EINVAL, "autotuning needs perspectives");
    nbt_ig_ctx* ctx = map->ctx;
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    VpLaunch L;
    float ms;
    int rc = launch_search(
        ctx->vp_launch, s, 2,
        [&](const VpLaunch& v) {
            nbt_ig_launch l = from_vp(v);
            return nbt_ig_ctx_set_launch(ctx, &l);
        },
        [&]() { return nbt_ig_eval_viewpoints(map, cam, poses, n, ig_out, steps_out, stream); }, &L, &ms);
    if (rc) return rc;
    *best = from_vp(L);
    *best_ms = ms;
    return NBT_IG_OK;
}

int nbt_ig_batch_autotune_layout(nbt_ig_batch* b, const uint32_t* vp_offsets, const float* poses,
                                 float* ig_out, uint64_t* steps_out, void* stream, int* best_layout,
                                 float* best_ms) {
    if (!b || !best_layout || !best_ms) return fail(NBT_IG_EINVAL, "batch, best_layout or best_ms is NULL");
    {
        std::lock_guard<std::mutex> lk(b->ctx->mu);
        for (nbt_ig_map* mk : b->maps)
            if (mk->batch_refs > 1) return fail(NBT_IG_EINVAL, "a map of this batch is held by another batch too");
    }
    DeviceGuard g(b->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", b->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    // every map in one order, then the descriptor table follows and the graph is rebuilt
    auto apply = [&](int lay) -> int {
        std::vector<DevMap> table(b->n_maps);
        for (uint32_t k = 0; k < b->n_maps; ++k) {
            if (int rc = relayout_map(b->maps[k], lay, s)) return rc;
            table[k] = b->maps[k]->dm;
        }
        hipError_t e = hipMemcpy(b->d_maps, table.data(), b->n_maps * sizeof(DevMap), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "batch descriptor table");
        drop_graph(b);
        return NBT_IG_OK;
    };
    const int start = b->maps.empty() ? NBT_IG_LAYOUT_LINEAR : b->maps[0]->dm.layout;
    float ms[kLayouts] = {};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    }
    int rc = NBT_IG_OK;
    for (int i = 0; i < kLayouts && rc == NBT_IG_OK; ++i) {
        const int lay = (start + i) % kLayouts;        // the current order first
        rc = apply(lay);
        if (rc == NBT_IG_OK) rc = nbt_ig_batch_run(b, vp_offsets, poses, ig_out, steps_out, stream);
        hipError_t e = rc == NBT_IG_OK ? hipEventRecord(e0, s) : hipSuccess;
        for (int r = 0; r < 3 && rc == NBT_IG_OK && e == hipSuccess; ++r)
            rc = nbt_ig_batch_run(b, vp_offsets, poses, ig_out, steps_out, stream);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventElapsedTime(&ms[lay], e0, e1);
        if (rc == NBT_IG_OK && e != hipSuccess) rc = hip_fail(e, "layout timing");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NBT_IG_OK) return rc;
    const int lay = fastest_layout(ms);
    if (int r2 = apply(lay)) return r2;
    *best_layout = lay;
    *best_ms = ms[lay] / 3.0f;
    return NBT_IG_OK;
}

int nbt_ig_autotune_trajectories(nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                 uint32_t n_traj, uint32_t poses_per_traj, float* ig_union, uint32_t* counts,
                                 uint64_t* visits, void* stream, int* best_layout, int* best_waves,
                                 float* best_ms) {
    if (int rc = check_map(map)) return rc;
    if (!best_layout || !best_waves || !best_ms) return fail(NBT_IG_EINVAL, "an output is NULL");
    if (n_traj == 0) return fail(NBT_IG_EINVAL, "autotuning needs trajectories");
    nbt_ig_ctx* ctx = map->ctx;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    }
    static const int waves[] = {4, 8, 16};
    float best = 0.0f;
    bool have = false;
    const int orig_waves = ctx->traj_waves;
    int bl = map->dm.layout, bw = orig_waves;
    int rc = NBT_IG_OK;
    const int start = map->dm.layout;
    for (int i = 0; i < kLayouts && rc == NBT_IG_OK; ++i) {
        const int lay = (start + i) % kLayouts;        // the current order first
        rc = nbt_ig_map_set_layout(map, lay, stream);
        for (int w = 0; w < 3 && rc == NBT_IG_OK; ++w) {
            rc = nbt_ig_ctx_set_traj_waves(ctx, waves[w]);
            if (rc == NBT_IG_OK)
                rc = nbt_ig_eval_trajectories(map, cam, poses, n_traj, poses_per_traj, ig_union, counts, visits,
                                              stream);
            hipError_t e = rc == NBT_IG_OK ? hipEventRecord(e0, s) : hipSuccess;
            for (int r = 0; r < 2 && rc == NBT_IG_OK && e == hipSuccess; ++r)
                rc = nbt_ig_eval_trajectories(map, cam, poses, n_traj, poses_per_traj, ig_union, counts, visits,
                                              stream);
            float ms = 0.0f;
            if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventRecord(e1, s);
            if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventSynchronize(e1);
            if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (rc == NBT_IG_OK && e != hipSuccess) rc = hip_fail(e, "trajectory timing");
            if (rc == NBT_IG_OK && (!have || ms < best)) {
                have = true;
                best = ms;
                bl = lay;
                bw = waves[w];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NBT_IG_OK) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->traj_waves = orig_waves;      // the map keeps whichever order it reached
        return rc;
    }
    if (int r2 = nbt_ig_map_set_layout(map, bl, stream)) return r2;
    if (int r2 = nbt_ig_ctx_set_traj_waves(ctx, bw)) return r2;
    *best_layout = bl;
    *best_waves = bw;
    *best_ms = best / 2.0f;
    return NBT_IG_OK;
}

int nbt_ig_autotune_map(nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses, uint32_t n,
                        float* ig_out, uint64_t* steps_out, void* stream, nbt_ig_launch* best,
                        int* best_layout, float* best_ms) {
    if (int rc = check_map(map)) return rc;
    if (!best || !best_layout || !best_ms) return fail(NBT_IG_EINVAL, "best, best_layout or best_ms is NULL");
    if (n == 0) return fail(NBT_IG_EINVAL, "autotuning needs perspectives");
    hipStream_t s = (hipStream_t)stream;
    // each layout at the context's current shape, then the shape search on the faster one
    const int start = map->dm.layout;
    float ms[kLayouts] = {};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBT_IG_EDEVICE, "hipEventCreate failed");
    }
    int rc = NBT_IG_OK;
    for (int i = 0; i < kLayouts && rc == NBT_IG_OK; ++i) {
        const int lay = (start + i) % kLayouts;        // the current order first
        rc = nbt_ig_map_set_layout(map, lay, stream);
        if (rc == NBT_IG_OK) rc = nbt_ig_eval_viewpoints(map, cam, poses, n, ig_out, steps_out, stream);
        hipError_t e = rc == NBT_IG_OK ? hipEventRecord(e0, s) : hipSuccess;
        for (int r = 0; r < 2 && rc == NBT_IG_OK && e == hipSuccess; ++r)
            rc = nbt_ig_eval_viewpoints(map, cam, poses, n, ig_out, steps_out, stream);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        if (rc == NBT_IG_OK && e == hipSuccess) e = hipEventElapsedTime(&ms[lay], e0, e1);
        if (rc == NBT_IG_OK && e != hipSuccess) rc = hip_fail(e, "layout timing");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NBT_IG_OK) return rc;
    const int lay = fastest_layout(ms);
    if (int r2 = nbt_ig_map_set_layout(map, lay, stream)) return r2;
    *best_layout = lay;
    return nbt_ig_autotune_viewpoints(map, cam, poses, n, ig_out, steps_out, stream, best, best_ms);
}

int nbt_ig_batch_autotune(nbt_ig_batch* b, const uint32_t* vp_offsets, const float* poses,
                          float* ig_out, uint64_t* steps_out, void* stream, nbt_ig_launch* best,
                          float* best_ms) {
    if (!b || !best || !best_ms) return fail(NBT_IG_EINVAL, "batch, best or best_ms is NULL");
    DeviceGuard g(b->ctx->device);
    VpLaunch L;
    float ms;
    int rc = launch_search(
        b->launch, (hipStream_t)stream, 3,
        [&](const VpLaunch& v) {
            nbt_ig_launch l = from_vp(v);
            return nbt_ig_batch_set_launch(b, &l);
        },
        [&]() { return nbt_ig_batch_run(b, vp_offsets, poses, ig_out, steps_out, stream); }, &L, &ms);
    if (rc) return rc;
    *best = from_vp(L);
    *best_ms = ms;
    return NBT_IG_OK;
}

}  // extern "C"
