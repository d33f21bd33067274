// RMSE and regularised loss over a COO rating set (Algorithm 1's stopping
// test and Section 5's reported test RMSE; Eq 4 and Eq 9).
//
// Each residual is formed in FP32 exactly as the training update forms it;
// squares and penalties are accumulated in FP64.  The work split is fixed
// (a fixed grid, rating t always handled by the same wave slot, partials
// combined by fixed trees), so the result is independent of timing.
#pragma clang fp contract(off)

#include <algorithm>

#include "internal.h"
#include "wave.h"

namespace bmf {

constexpr int EV_WG = 256;
constexpr int EV_GRID = 1024;
constexpr int EV_WAVES = EV_WG / WAVE;
// 16 lanes per rating, 4 ratings per wave step; lane owns factors
// 4*(lane%16) + 64*c .. +3.
constexpr int LPR = 16;

template <int KV>  // float4 vectors per lane: k <= 64*KV
__global__ __launch_bounds__(EV_WG) void sqres_kernel(const int32_t *__restrict__ u, const int32_t *__restrict__ i,
                                                      const float *__restrict__ r, int64_t cnt, int k,
                                                      const float *__restrict__ P, const float *__restrict__ Q,
                                                      const float *__restrict__ bu, const float *__restrict__ bi,
                                                      float mu, int with_penalty, HP hp, double *__restrict__ part) {
    __shared__ double sh[EV_WG];
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    const int sub = lane / LPR, sl = lane % LPR;
    const int64_t slot = ((int64_t)blockIdx.x * EV_WAVES + wave) * 4 + sub;
    const int64_t nslots = (int64_t)EV_GRID * EV_WAVES * 4;
    double acc = 0.0;
    for (int64_t t = slot; t < cnt; t += nslots) {
        const int64_t uu = u[t], ii = i[t];
        float d = 0.f;
        double pp = 0.0, qq = 0.0;
        bool first = true;
#pragma unroll
        for (int c = 0; c < KV; ++c) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int f = 64 * c + 4 * sl + e;
                const float pv = f < k ? P[uu * k + f] : 0.f;
                const float qv = f < k ? Q[ii * k + f] : 0.f;
                d = first ? pv * qv : fmaf(pv, qv, d);
                first = false;
                pp += (double)pv * pv;
                qq += (double)qv * qv;
            }
        }
        // sum over the 16 lanes of this rating (fixed butterfly)
        d = row16_sum(d);
        const float bu0 = bu[uu], bi0 = bi[ii];
        const float e = (((r[t] - mu) - bu0) - bi0) - d;
        if (sl == 0) {
            double v = (double)e * (double)e;
            acc += v;
        }
        if (with_penalty) {
            // penalties: lane-partials in FP64, reduced over the 16 lanes
            for (int off = 1; off < LPR; off <<= 1) {
                pp += __shfl_xor(pp, off, WAVE);
                qq += __shfl_xor(qq, off, WAVE);
            }
            if (sl == 0)
                acc += (double)hp.b_p * pp + (double)hp.b_q * qq + (double)hp.b_bu * ((double)bu0 * bu0) +
                       (double)hp.b_bi * ((double)bi0 * bi0);
        }
    }
    // combine the slots of the workgroup in a fixed tree
    sh[tid] = (sl == 0) ? acc : 0.0;
    __syncthreads();
    for (int w = EV_WG / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(EV_WG) void sum_parts_kernel(const double *__restrict__ part, int n,
                                                          double *__restrict__ out) {
    __shared__ double sh[EV_WG];
    double a = 0.0;
    for (int t = threadIdx.x; t < n; t += EV_WG) a += part[t];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = EV_WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

double sq_residual_sum(const Model &M, const int32_t *u, const int32_t *i, const float *r, int64_t cnt,
                       const HP *loss_hp, DevBuf &scratch) {
    if (cnt == 0) return 0.0;
    const size_t need = (EV_GRID + 1) * sizeof(double);
    if (scratch.bytes < need) scratch.alloc(std::max<size_t>(need, 1 << 16));
    double *part = scratch.as<double>();
    const int kv = (M.k + 63) / 64;
    HP hp = loss_hp ? *loss_hp : HP{0, 0, 0, 0, 0, 0, 0, 0};
    const int pen = loss_hp ? 1 : 0;
    const float mu = (float)M.mu;
#define EV_LAUNCH(KV)                                                                                        \
    sqres_kernel<KV><<<EV_GRID, EV_WG, 0, M.stream>>>(u, i, r, cnt, M.k, M.P.as<float>(), M.Q.as<float>(),   \
                                                      M.bu.as<float>(), M.bi.as<float>(), mu, pen, hp, part)
    switch (kv) {
    case 1: EV_LAUNCH(1); break;
    case 2: EV_LAUNCH(2); break;
    case 3: EV_LAUNCH(3); break;
    case 4: EV_LAUNCH(4); break;
    case 5: case 6: case 7: case 8: EV_LAUNCH(8); break;
    default: EV_LAUNCH(16); break;
    }
#undef EV_LAUNCH
    BMF_HIP(hipGetLastError());
    sum_parts_kernel<<<1, EV_WG, 0, M.stream>>>(part, EV_GRID, part + EV_GRID);
    BMF_HIP(hipGetLastError());
    double out = 0.0;
    BMF_HIP(hipMemcpyAsync(&out, part + EV_GRID, sizeof(double), hipMemcpyDeviceToHost, M.stream));
    BMF_HIP(hipStreamSynchronize(M.stream));
    return out;
}

}  // namespace bmf
