// cost.hip -- planner-side IG terms of Sec. IV for many candidate horizons.
//
//   G(x)  Eq. 3: inverse-distance weighting of the perspectives' IG, summed
//         over the N_B buffered information distributions with weight
//         1/(N_B - u) (u = 0 oldest);
//   O(x)  cosine between the camera's viewing axis and the direction to the
//         PoI, 0 when the PoI is outside the field of view;
//   c_I   sum over a horizon's states of w_I / (O G + eps).
// One thread per horizon state; perspectives stream through LDS in tiles
// that every thread of the block reads (broadcast).  ALU-bound: ~12 VALU
// operations per (state, perspective) pair.
#include "internal.hpp"

namespace nbt {

constexpr int kCostTile = 256;

__global__ __launch_bounds__(256) void idw_query_kernel(const float* __restrict__ id_pos,
                                                        const float* __restrict__ id_ig, uint32_t nb,
                                                        uint32_t np, float p, const float* __restrict__ poses,
                                                        uint32_t q_count, float px, float py, float pz,
                                                        float tan_h, float tan_v, float* __restrict__ g_out,
                                                        float* __restrict__ o_out) {
    __shared__ float4 tile[kCostTile];
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = q < q_count;
    float tx = 0.0f, ty = 0.0f, tz = 0.0f;
    if (active) {
        tx = poses[12 * (size_t)q + 9];
        ty = poses[12 * (size_t)q + 10];
        tz = poses[12 * (size_t)q + 11];
    }
    const bool p_two = (p == 2.0f);
    const float half_neg_p = -0.5f * p;
    double g_sum = 0.0;
    for (uint32_t u = 0; u < nb; ++u) {
        double num = 0.0, den = 0.0, num0 = 0.0;
        uint32_t cnt0 = 0;
        for (uint32_t j0 = 0; j0 < np; j0 += kCostTile) {
            __syncthreads();
            const uint32_t j = j0 + threadIdx.x;
            if (j < np) {
                const size_t s = (size_t)u * np + j;
                tile[threadIdx.x] = make_float4(id_pos[3 * s], id_pos[3 * s + 1], id_pos[3 * s + 2], id_ig[s]);
            }
            __syncthreads();
            const uint32_t len = (np - j0) < (uint32_t)kCostTile ? (np - j0) : (uint32_t)kCostTile;
            float fnum = 0.0f, fden = 0.0f;
            for (uint32_t k = 0; k < len; ++k) {
                const float4 e = tile[k];
                const float dx = e.x - tx, dy = e.y - ty, dz = e.z - tz;
                const float d2 = dx * dx + dy * dy + dz * dz;
                if (dx == 0.0f && dy == 0.0f && dz == 0.0f) {
                    num0 += (double)e.w;
                    ++cnt0;
                } else {
                    const float w = p_two ? __builtin_amdgcn_rcpf(d2) : __builtin_powf(d2, half_neg_p);
                    fnum += e.w * w;
                    fden += w;
                }
            }
            num += (double)fnum;
            den += (double)fden;
        }
        const double g_u = cnt0 ? num0 / (double)cnt0 : num / den;
        g_sum += g_u / (double)(nb - u);
    }
    if (!active) return;
    g_out[q] = (float)g_sum;
    // orientation factor: camera coordinates of the PoI, c = R^T (poi - t)
    const float* r = poses + 12 * (size_t)q;
    const float vx = px - tx, vy = py - ty, vz = pz - tz;
    const float cx = r[0] * vx + r[3] * vy + r[6] * vz;
    const float cy = r[1] * vx + r[4] * vy + r[7] * vz;
    const float cz = r[2] * vx + r[5] * vy + r[8] * vz;
    const float n = sqrtf(vx * vx + vy * vy + vz * vz);
    float o = 0.0f;
    if (cz > 0.0f && n > 0.0f && fabsf(cx / cz) <= tan_h && fabsf(cy / cz) <= tan_v) o = cz / n;
    o_out[q] = o;
}

__global__ __launch_bounds__(256) void horizon_cost_kernel(const float* __restrict__ g,
                                                           const float* __restrict__ o, uint32_t h,
                                                           uint32_t k, float w_i, float eps,
                                                           float* __restrict__ cost) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h) return;
    double s = 0.0;
    for (uint32_t j = 0; j < k; ++j) {
        const size_t q = (size_t)i * k + j;
        s += (double)w_i / ((double)o[q] * (double)g[q] + (double)eps);
    }
    cost[i] = (float)s;
}

hipError_t launch_eval_cost(const float* id_pos, const float* id_ig, uint32_t nb, uint32_t np, float p,
                            const float* poses, uint32_t h, uint32_t k, const float poi[3], float tan_h,
                            float tan_v, float w_i, float eps, float* g_out, float* o_out, float* cost,
                            hipStream_t s) {
    const uint32_t q = h * k;
    hipLaunchKernelGGL(idw_query_kernel, dim3((q + 255) / 256), dim3(256), 0, s, id_pos, id_ig, nb, np, p,
                       poses, q, poi[0], poi[1], poi[2], tan_h, tan_v, g_out, o_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !cost) return e;
    hipLaunchKernelGGL(horizon_cost_kernel, dim3((h + 255) / 256), dim3(256), 0, s, g_out, o_out, h, k, w_i,
                       eps, cost);
    return hipGetLastError();
}

}  // namespace nbt
