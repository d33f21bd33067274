// Folding-in of new users (the projection of new data onto a trained model
// that Section 2.1 cites and Section 6 proposes for incremental data):
// item factors and biases stay fixed, the new user's p and bu start at zero
// and take `passes` passes of the user-side updates (Eq 10 and Eq 12) over
// the user's ratings in input order.
//
// One workgroup per request.  All four waves stage the request's item rows
// and biases into LDS (as many rows as fit); wave 0 then runs the dependent
// chain with p in registers (lane f owns factors f, f+64, ...), reading the
// next row one rating ahead.  Rows that did not fit are read from global
// memory with the same one-ahead prefetch (Q is read-only here, so every
// prefetch is valid).
#pragma clang fp contract(off)

#include <algorithm>

#include "internal.h"
#include "wave.h"

namespace bmf {

constexpr int FI_WG = 256;

template <int KPL>
__global__ __launch_bounds__(FI_WG) void foldin_kernel(const int32_t *__restrict__ items, const float *__restrict__ r,
                                                       const int64_t *__restrict__ off, int passes,
                                                       const float *__restrict__ Q, const float *__restrict__ bi,
                                                       int k, float mu, HP hp, int stage_rows,
                                                       float *__restrict__ p_out, float *__restrict__ bu_out,
                                                       int64_t p_stride) {
    extern __shared__ __align__(16) float fsm[];
    const int64_t req = blockIdx.x;
    const int64_t beg = off[req];
    const int cnt = (int)(off[req + 1] - beg);
    const int rows = std::min(cnt, stage_rows);
    float *qs = fsm;                      // rows * k
    float *bs = fsm + (size_t)rows * k;   // rows
    float *rs = bs + rows;                // rows
    const int tid = threadIdx.x;
    for (int64_t x = tid; x < (int64_t)rows * k; x += FI_WG) {
        const int j = (int)(x / k), f = (int)(x % k);
        qs[x] = Q[(int64_t)items[beg + j] * k + f];
    }
    for (int j = tid; j < rows; j += FI_WG) {
        bs[j] = bi[items[beg + j]];
        rs[j] = r[beg + j];
    }
    __syncthreads();
    if (tid >= WAVE) return;
    const int lane = tid;
    float p[KPL];
#pragma unroll
    for (int c = 0; c < KPL; ++c) p[c] = 0.f;
    float bu = 0.f;
    auto load = [&](int j, float (&q)[KPL], float &b, float &rv) {
        if (j < rows) {
#pragma unroll
            for (int c = 0; c < KPL; ++c) {
                const int f = lane + WAVE * c;
                q[c] = f < k ? qs[(size_t)j * k + f] : 0.f;
            }
            b = bs[j];
            rv = rs[j];
        } else {
            const int64_t it = items[beg + j];
#pragma unroll
            for (int c = 0; c < KPL; ++c) {
                const int f = lane + WAVE * c;
                q[c] = f < k ? Q[it * k + f] : 0.f;
            }
            b = bi[it];
            rv = r[beg + j];
        }
    };
    if (cnt > 0) {
        float qn[KPL], bn, rn;
        load(0, qn, bn, rn);
        for (int pass = 0; pass < passes; ++pass) {
            for (int j = 0; j < cnt; ++j) {
                float q[KPL];
#pragma unroll
                for (int c = 0; c < KPL; ++c) q[c] = qn[c];
                const float b0 = bn, rv = rn;
                const int jn = (j + 1 < cnt) ? j + 1 : 0;
                load(jn, qn, bn, rn);
                float d = p[0] * q[0];
#pragma unroll
                for (int c = 1; c < KPL; ++c) d = fmaf(p[c], q[c], d);
                d = wave_sum_dpp(d);
                const float e = (((rv - mu) - bu) - b0) - d;
                bu = fmaf(hp.a_bu, fmaf(-hp.b_bu, bu, e), bu);
#pragma unroll
                for (int c = 0; c < KPL; ++c) p[c] = fmaf(hp.a_p, fmaf(e, q[c], -(hp.b_p * p[c])), p[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
        const int f = lane + WAVE * c;
        if (f < k) p_out[req * p_stride + f] = p[c];
    }
    if (lane == 0) bu_out[req] = bu;
}

static int max_lds(int device) {
    int v = 0;
    BMF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    return v;
}

void foldin_launch(Model &M, const int32_t *d_items, const float *d_r, const int64_t *d_off, int64_t nreq,
                   int max_cnt, int passes, const HP &hp, float *d_p, int64_t p_stride, float *d_bu, hipStream_t s) {
    if (nreq == 0) return;
    static int lds_cap = 0;
    if (!lds_cap) lds_cap = max_lds(M.device);
    const int row_bytes = M.k * 4 + 8;
    const int stage_rows = std::max(0, std::min(max_cnt, (lds_cap - 256) / row_bytes));
    const size_t lds = (size_t)stage_rows * row_bytes;
    const int kpl = (M.k + WAVE - 1) / WAVE;
#define FI_LAUNCH(KPL)                                                                                            \
    do {                                                                                                          \
        BMF_HIP(hipFuncSetAttribute((const void *)foldin_kernel<KPL>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                    lds_cap));                                                                    \
        foldin_kernel<KPL><<<(unsigned)nreq, FI_WG, lds, s>>>(d_items, d_r, d_off, passes, M.Q.as<float>(),         \
                                                                     M.bi.as<float>(), M.k, (float)M.mu, hp,      \
                                                                     stage_rows, d_p, d_bu, p_stride);            \
    } while (0)
    switch (kpl) {
    case 1: FI_LAUNCH(1); break;
    case 2: FI_LAUNCH(2); break;
    case 3: FI_LAUNCH(3); break;
    case 4: FI_LAUNCH(4); break;
    default: FI_LAUNCH(16); break;
    }
#undef FI_LAUNCH
    BMF_HIP(hipGetLastError());
}

void foldin_run(Model &M, const int32_t *d_items, const float *d_r, int nr, int passes, const HP &hp, float *d_p,
                float *d_bu) {
    DevBuf off;
    off.alloc(2 * sizeof(int64_t));
    const int64_t h[2] = {0, nr};
    BMF_HIP(hipMemcpyAsync(off.p, h, sizeof(h), hipMemcpyHostToDevice, M.stream));
    foldin_launch(M, d_items, d_r, off.as<int64_t>(), 1, nr, passes, hp, d_p, M.k, d_bu, M.stream);
    BMF_HIP(hipStreamSynchronize(M.stream));
}

__device__ __forceinline__ uint16_t bf16_rne_bits(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__global__ void foldin_rows_kernel(const float *__restrict__ bu_f, int64_t nreq, float mu, int k, int kp, int kb,
                                   float *__restrict__ Ug, uint16_t *__restrict__ Ugb, float *__restrict__ ub) {
    const int64_t total = nreq * kb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / kb;
        const int f = (int)(t % kb);
        float v = 0.f;
        if (f < k) v = Ug[q * kp + f];
        else if (f < kp) Ug[q * kp + f] = 0.f;
        if (Ugb) Ugb[q * kb + f] = bf16_rne_bits(v);
        if (f == 0) ub[q] = mu + bu_f[q];
    }
}

void foldin_rows(const float *bu_f, int64_t nreq, float mu, int k, int kp, int kb, float *Ug, uint16_t *Ugb,
                 float *ub, hipStream_t s) {
    if (nreq == 0) return;
    const int grid = (int)std::min<int64_t>((nreq * kb + 255) / 256, 4096);
    foldin_rows_kernel<<<grid, 256, 0, s>>>(bu_f, nreq, mu, k, kp, kb, Ug, Ugb, ub);
    BMF_HIP(hipGetLastError());
}

}  // namespace bmf
