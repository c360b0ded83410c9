// surrogate_api.hip -- host side of the learned IG surrogate.
#include <vector>

#include "host.hpp"
#include "surrogate.hpp"

using namespace nbt;

namespace {

uint16_t to_bf16(float f) {                       // round to nearest, ties to even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

struct nbt_ig_surrogate {
    nbt_ig_ctx* ctx = nullptr;
    float extent = 0, dist_mean = 0, dist_scale = 1, out_scale = 1, b3 = 0;
    int kpad[4] = {0, 0, 0, 0};
    __bf16* conv_w[4] = {nullptr, nullptr, nullptr, nullptr};
    float* conv_b[4] = {nullptr, nullptr, nullptr, nullptr};
    __bf16* w1f = nullptr;
    float* w1d = nullptr;
    float* b1 = nullptr;
    __bf16* w2 = nullptr;
    float* b2 = nullptr;
    float* w3 = nullptr;
    // per-call buffers
    __bf16* act2 = nullptr;      // conv2 output, channel-last
    __bf16* act3 = nullptr;      // conv3 output, channel-last
    __bf16* feat = nullptr;      // trunk features
    __bf16* patch = nullptr;     // the counted patch, for cells wider than the trunk counts itself
    float* c = nullptr;
    float* pred = nullptr;       // predictions of a selection (grown stream-ordered)
    size_t pred_bytes = 0;
    bool pred_async = false;
    uint32_t* sel = nullptr;     // selection stages' keys and indices (grown stream-ordered)
    size_t sel_bytes = 0;
    bool sel_async = false;
    uint32_t* cand = nullptr;
    float* cand_poses = nullptr;
    float* cand_ig = nullptr;
    std::vector<void*> owned;
};

namespace {

template <class T>
hipError_t dalloc(nbt_ig_surrogate* s, T** p, size_t count) {
    hipError_t e = hipMalloc(p, count * sizeof(T));
    if (e == hipSuccess) s->owned.push_back((void*)*p);
    return e;
}

template <class T>
hipError_t upload(nbt_ig_surrogate* s, T** p, const std::vector<T>& host) {
    hipError_t e = dalloc(s, p, host.size());
    if (e == hipSuccess) e = hipMemcpy(*p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int run_trunk(nbt_ig_surrogate* s, const nbt_ig_map* map, const float poi[3], float* patch_f32,
              hipStream_t st) {
    const double vox = map->voxel;
    const double fd = std::floor((double)s->extent / (kGrid * vox) + 0.5);
    if (!(fd <= 4096.0)) return fail(NBT_IG_EUNSUPPORTED, "patch extent of more than 4096 voxels per cell");
    const int f = fd < 1.0 ? 1 : (int)fd;
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        const double q = std::floor(((double)poi[a] - (double)map->origin[a]) / vox + 0.5);
        if (!(std::fabs(q) < 1e9)) return fail(NBT_IG_EINVAL, "PoI is not finite or too far from the map");
        i0[a] = (int)q - (kGrid / 2) * f;
    }
    hipError_t e = hipSuccess;
    const bool counted = f > kFrontCountMaxF;
    if (patch_f32 || counted) e = launch_patch(map->dm, f, i0, counted ? s->patch : nullptr, patch_f32, st);
    if (e == hipSuccess) {
        TrunkArgs a;
        a.m = map->dm;
        a.f = f;
        a.i0x = i0[0];
        a.i0y = i0[1];
        a.i0z = i0[2];
        a.patch = counted ? s->patch : nullptr;
        for (int l = 0; l < 4; ++l) {
            a.w[l] = s->conv_w[l];
            a.b[l] = s->conv_b[l];
        }
        a.w1f = s->w1f;
        a.fb1 = s->b1;
        a.act2 = s->act2;
        a.act3 = s->act3;
        a.feat = s->feat;
        a.c = s->c;
        e = launch_trunk(a, st);
    }
    if (e != hipSuccess) return hip_fail(e, "surrogate trunk");
    return NBT_IG_OK;
}

int check_poi(const float poi[3]) {
    if (!poi || !std::isfinite(poi[0]) || !std::isfinite(poi[1]) || !std::isfinite(poi[2]))
        return fail(NBT_IG_EINVAL, "poi must be 3 finite floats");
    return NBT_IG_OK;
}

}  // namespace

extern "C" {

int nbt_ig_surrogate_create(nbt_ig_ctx* ctx, const void* weights, size_t nbytes, nbt_ig_surrogate** out) {
    if (!out) return fail(NBT_IG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !weights) return fail(NBT_IG_EINVAL, "ctx or weights is NULL");
    size_t expect = 32;
    for (int l = 0; l < 4; ++l) expect += 4 * ((size_t)kConvOut[l] * kConvIn[l] * 27 + kConvOut[l]);
    expect += 4 * ((size_t)kHidden * (kFeat + 4) + kHidden + (size_t)kHidden * kHidden + kHidden + kHidden + 1);
    const unsigned char* b = static_cast<const unsigned char*>(weights);
    uint32_t version = 0;
    if (nbytes >= 8) std::memcpy(&version, b + 4, 4);
    if (nbytes != expect || std::memcmp(b, "NBTS", 4) != 0 || version != 1)
        return fail(NBT_IG_EINVAL, "weights blob: expected NBTS version 1 of %zu bytes, got %zu bytes", expect, nbytes);
    float meta[4];
    std::memcpy(meta, b + 8, sizeof meta);
    if (!finite_pos(meta[0]) || !std::isfinite(meta[1]) || !finite_pos(meta[2]) || !std::isfinite(meta[3]))
        return fail(NBT_IG_EINVAL, "weights blob: bad extent or normalisation constants");
    std::vector<float> p((expect - 32) / 4);
    std::memcpy(p.data(), b + 32, expect - 32);
    for (float v : p)
        if (!std::isfinite(v)) return fail(NBT_IG_EINVAL, "weights blob holds non-finite values");

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    nbt_ig_surrogate* s = new (std::nothrow) nbt_ig_surrogate;
    if (!s) return fail(NBT_IG_ENOMEM, "host allocation failed");
    s->ctx = ctx;
    s->extent = meta[0];
    s->dist_mean = meta[1];
    s->dist_scale = meta[2];
    s->out_scale = meta[3];
    hipError_t e = hipSuccess;
    size_t off = 0;
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
        // blob order [cout][cin][tap]; library order k = ci*27 + tap for conv1,
        // k = tap*cin + ci for the others (see TrunkArgs)
        const int ci = kConvIn[l], co = kConvOut[l], K = ci * 27;
        s->kpad[l] = conv_kpad(l);
        std::vector<uint16_t> w((size_t)co * s->kpad[l], 0);
        for (int n = 0; n < co; ++n)
            for (int c = 0; c < ci; ++c)
                for (int tap = 0; tap < 27; ++tap) {
                    const int k = l == 0 ? c * 27 + tap : tap * ci + c;
                    w[(size_t)n * s->kpad[l] + k] = to_bf16(p[off + (size_t)n * K + (size_t)c * 27 + tap]);
                }
        off += (size_t)co * K;
        std::vector<float> bias(p.begin() + off, p.begin() + off + co);
        off += co;
        e = upload(s, reinterpret_cast<uint16_t**>(&s->conv_w[l]), w);
        if (e == hipSuccess) e = upload(s, &s->conv_b[l], bias);
    }
    if (e == hipSuccess) {
        std::vector<uint16_t> w1f((size_t)kHidden * kFeat);
        std::vector<float> w1d((size_t)kHidden * 4);
        for (int n = 0; n < kHidden; ++n) {
            for (int k = 0; k < kFeat; ++k) w1f[(size_t)n * kFeat + k] = to_bf16(p[off + (size_t)n * (kFeat + 4) + k]);
            for (int k = 0; k < 4; ++k) w1d[(size_t)n * 4 + k] = p[off + (size_t)n * (kFeat + 4) + kFeat + k];
        }
        off += (size_t)kHidden * (kFeat + 4);
        std::vector<float> b1(p.begin() + off, p.begin() + off + kHidden);
        off += kHidden;
        // W2 with its columns in the order the MLP kernel builds h1 in registers:
        // stored position j holds neuron j with bits 2 and 3 of its index swapped
        std::vector<uint16_t> w2((size_t)kHidden * kHidden);
        for (int n = 0; n < kHidden; ++n)
            for (int j = 0; j < kHidden; ++j) {
                const int src = (j & ~0xC) | ((j & 4) << 1) | ((j & 8) >> 1);
                w2[(size_t)n * kHidden + j] = to_bf16(p[off + (size_t)n * kHidden + src]);
            }
        off += w2.size();
        std::vector<float> b2(p.begin() + off, p.begin() + off + kHidden);
        off += kHidden;
        std::vector<float> w3(p.begin() + off, p.begin() + off + kHidden);
        off += kHidden;
        s->b3 = p[off];
        e = upload(s, reinterpret_cast<uint16_t**>(&s->w1f), w1f);
        if (e == hipSuccess) e = upload(s, &s->w1d, w1d);
        if (e == hipSuccess) e = upload(s, &s->b1, b1);
        if (e == hipSuccess) e = upload(s, reinterpret_cast<uint16_t**>(&s->w2), w2);
        if (e == hipSuccess) e = upload(s, &s->b2, b2);
        if (e == hipSuccess) e = upload(s, &s->w3, w3);
    }
    if (e == hipSuccess) e = dalloc(s, &s->act2, (size_t)kConvOut[1] * 8 * 8 * 8);
    if (e == hipSuccess) e = dalloc(s, &s->act3, (size_t)kConvOut[2] * 4 * 4 * 4);
    if (e == hipSuccess) e = dalloc(s, &s->feat, kFeat);
    if (e == hipSuccess) e = dalloc(s, &s->patch, 2 * (size_t)kPatchCells);
    if (e == hipSuccess) e = dalloc(s, &s->c, kHidden);
    if (e == hipSuccess) e = dalloc(s, &s->cand, kMaxRescore);
    if (e == hipSuccess) e = dalloc(s, &s->cand_poses, 12 * (size_t)kMaxRescore);
    if (e == hipSuccess) e = dalloc(s, &s->cand_ig, kMaxRescore);
    if (e != hipSuccess) {
        nbt_ig_surrogate_destroy(s);
        return hip_fail(e, "surrogate upload");
    }
    *out = s;
    return NBT_IG_OK;
}

void nbt_ig_surrogate_destroy(nbt_ig_surrogate* s) {
    if (!s) return;
    DeviceGuard g(s->ctx->device);
    for (void* p : s->owned) (void)hipFree(p);
    release_buffer(s->pred, s->pred_async, nullptr);
    release_buffer(s->sel, s->sel_async, nullptr);
    if (s->pred_async || s->sel_async) (void)hipStreamSynchronize(nullptr);
    delete s;
}

int nbt_ig_surrogate_predict(nbt_ig_surrogate* s, const nbt_ig_map* map, const float poi[3],
                             const float* poses, uint32_t n, float* pred, void* stream) {
    if (!s) return fail(NBT_IG_EINVAL, "surrogate is NULL");
    if (int rc = check_map(map)) return rc;
    if (map->ctx != s->ctx) return fail(NBT_IG_EINVAL, "map and surrogate belong to different contexts");
    if (int rc = check_poi(poi)) return rc;
    if (n == 0) return NBT_IG_OK;
    if (!poses || !pred) return fail(NBT_IG_EINVAL, "poses or pred is NULL");
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", s->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc = run_trunk(s, map, poi, nullptr, st)) return rc;
    hipError_t e = launch_mlp(poses, n, poi, s->dist_mean, s->dist_scale, s->c, s->w1d, s->w2, s->b2, s->w3,
                              s->b3, s->out_scale, pred, s->ctx->cu_count, st);
    if (e != hipSuccess) return hip_fail(e, "surrogate mlp");
    return NBT_IG_OK;
}

int nbt_ig_surrogate_select(nbt_ig_surrogate* s, const nbt_ig_map* map, const nbt_ig_camera* cam,
                            const float poi[3], const float* poses, uint32_t n, uint32_t k_rescore,
                            uint32_t k, uint32_t* idx_out, float* ig_out, void* stream) {
    if (!s) return fail(NBT_IG_EINVAL, "surrogate is NULL");
    if (k < 1 || k > k_rescore || k_rescore > (uint32_t)kMaxRescore)
        return fail(NBT_IG_EINVAL, "need 1 <= k <= k_rescore <= %d", kMaxRescore);
    if (n < k_rescore || n > kMaxCandidates)
        return fail(NBT_IG_EUNSUPPORTED, "need k_rescore <= n <= 2^22 candidates (got %u)", n);
    if (!idx_out || !ig_out) return fail(NBT_IG_EINVAL, "idx_out or ig_out is NULL");
    CamParams cp;
    if (int rc = check_camera(cam, &cp)) return rc;
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", s->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (!poses) return fail(NBT_IG_EINVAL, "poses is NULL");
    if (int rc = check_map(map)) return rc;
    if (map->ctx != s->ctx) return fail(NBT_IG_EINVAL, "map and surrogate belong to different contexts");
    if (int rc = check_poi(poi)) return rc;
    {
        std::lock_guard<std::mutex> lk(s->ctx->mu);
        void* q = s->pred;
        if (int rc = grow_buffer(&q, &s->pred_bytes, &s->pred_async, (size_t)n * sizeof(float), st,
                                 "surrogate predictions"))
            return rc;
        s->pred = static_cast<float*>(q);
        const size_t items = select_scratch_items(n, k_rescore);
        if (items) {
            q = s->sel;
            if (int rc = grow_buffer(&q, &s->sel_bytes, &s->sel_async, 4 * items * sizeof(uint32_t), st,
                                     "surrogate selection stages"))
                return rc;
            s->sel = static_cast<uint32_t*>(q);
        }
    }
    // trunk, MLP, selection of the k_rescore best as a set with their poses,
    // exact rescoring, final pick
    if (int rc = run_trunk(s, map, poi, nullptr, st)) return rc;
    hipError_t e = launch_mlp(poses, n, poi, s->dist_mean, s->dist_scale, s->c, s->w1d, s->w2, s->b2, s->w3,
                              s->b3, s->out_scale, s->pred, s->ctx->cu_count, st);
    if (e == hipSuccess)
        e = launch_select(s->pred, n, k_rescore, poses, s->sel, select_scratch_items(n, k_rescore), s->cand,
                          s->cand_poses, st);
    if (e != hipSuccess) return hip_fail(e, "surrogate mlp and selection");
    if (int rc = nbt_ig_eval_viewpoints(map, cam, s->cand_poses, k_rescore, s->cand_ig, nullptr, stream))
        return rc;
    e = launch_final_select(s->cand_ig, s->cand, k_rescore, k, false, idx_out, ig_out, st);
    if (e != hipSuccess) return hip_fail(e, "surrogate select");
    return NBT_IG_OK;
}

int nbt_ig_surrogate_features(nbt_ig_surrogate* s, const nbt_ig_map* map, const float poi[3],
                              float* patch_out, float* features_out, void* stream) {
    if (!s) return fail(NBT_IG_EINVAL, "surrogate is NULL");
    if (int rc = check_map(map)) return rc;
    if (int rc = check_poi(poi)) return rc;
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", s->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (int rc = run_trunk(s, map, poi, patch_out, st)) return rc;
    if (features_out) {
        hipError_t e = launch_bf16_to_f32(s->feat, kFeat, features_out, st);
        if (e != hipSuccess) return hip_fail(e, "surrogate features");
    }
    return NBT_IG_OK;
}

int nbt_ig_top_k(nbt_ig_ctx* ctx, const float* values, uint32_t n, uint32_t k, uint32_t* idx_out,
                 float* val_out, void* stream) {
    if (!ctx) return fail(NBT_IG_EINVAL, "ctx is NULL");
    if (k < 1 || k > (uint32_t)kMaxRescore || n < k || n > kMaxCandidates)
        return fail(NBT_IG_EINVAL, "need 1 <= k <= %d and k <= n <= 2^22", kMaxRescore);
    if (!values || !idx_out) return fail(NBT_IG_EINVAL, "values or idx_out is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // the radix selection's stage buffers, then the chosen set (k indices)
    const size_t items = select_scratch_items(n, k);
    const size_t need = (4 * items + k) * sizeof(uint32_t);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        void* p = ctx->topk_keep;
        if (int rc = grow_buffer(&p, &ctx->topk_bytes, &ctx->topk_async, need, st, "top-k scratch")) return rc;
        ctx->topk_keep = static_cast<unsigned long long*>(p);
    }
    uint32_t* scratch = reinterpret_cast<uint32_t*>(ctx->topk_keep);
    uint32_t* set = scratch + 4 * items;
    hipError_t e = launch_select(values, n, k, nullptr, scratch, items, set, nullptr, st);
    if (e == hipSuccess) e = launch_final_select(values, set, k, k, true, idx_out, val_out, st);
    if (e != hipSuccess) return hip_fail(e, "top-k");
    return NBT_IG_OK;
}

int nbt_ig_extract_patch(const nbt_ig_map* map, const float poi[3], float extent, float* out, void* stream) {
    if (int rc = check_map(map)) return rc;
    if (int rc = check_poi(poi)) return rc;
    if (!finite_pos(extent) || !out) return fail(NBT_IG_EINVAL, "extent must be > 0 and out non-NULL");
    DeviceGuard g(map->ctx->device);
    if (!g.ok) return fail(NBT_IG_EDEVICE, "cannot select device %d", map->ctx->device);
    const double vox = map->voxel;
    int f = (int)std::floor((double)extent / (kGrid * vox) + 0.5);
    if (f < 1) f = 1;
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        const double q = std::floor(((double)poi[a] - (double)map->origin[a]) / vox + 0.5);
        if (!(std::fabs(q) < 1e9)) return fail(NBT_IG_EINVAL, "PoI too far from the map");
        i0[a] = (int)q - (kGrid / 2) * f;
    }
    hipError_t e = launch_patch(map->dm, f, i0, nullptr, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "patch_kernel");
    return NBT_IG_OK;
}

}  // extern "C"
