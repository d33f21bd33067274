// Stratified block SGD (Algorithm 1's epoch loop with Algorithm 2 as the
// per-block kernel; Eqs 10-13 as the per-rating update).
//
// One stratum s = {((j + s) mod b, j) : j < b} is one launch: workgroup j
// owns block ((j + s) mod b, j).  Blocks of a stratum share no block row and
// no block column (Section 3, parallel BMF), so the workgroups touch
// disjoint rows of P/bu and of Q/bi; the stream order between launches is
// the barrier between strata.
//
// Inside a block one wavefront walks the ratings in (u, i, t) order; lane f
// owns latent factors f, f + 64, ... .  Every variant below performs the
// same floating-point operations in the same order (rating_update), so all
// variants produce identical bits.
#pragma clang fp contract(off)

#include <algorithm>

#include "internal.h"
#include "wave.h"

namespace bmf {

// Dot-product partial of one lane: p[0]*q[0], then fma over the rest.
template <int KPL>
__device__ __forceinline__ float lane_dot(const float (&p)[KPL], const float (&q)[KPL]) {
    float d = p[0] * q[0];
#pragma unroll
    for (int c = 1; c < KPL; ++c) d = fmaf(p[c], q[c], d);
    return d;
}

// Eqs 10-13, one residual from pre-update values, explicit FMAs so that
// every kernel rounds identically:
//   g = err*other - beta*self (one fma, beta*self rounded first)
//   self' = self + alpha*g     (one fma)
template <int KPL>
__device__ __forceinline__ void factor_update(float (&p)[KPL], float (&q)[KPL], float e, const HP &hp) {
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
        const float pc = p[c], qc = q[c];
        const float gp = fmaf(e, qc, -(hp.b_p * pc));
        const float gq = fmaf(e, pc, -(hp.b_q * qc));
        p[c] = fmaf(hp.a_p, gp, pc);
        q[c] = fmaf(hp.a_q, gq, qc);
    }
}

__device__ __forceinline__ float bias_update(float b0, float e, float a, float beta) {
    return fmaf(a, fmaf(-beta, b0, e), b0);
}

__device__ __forceinline__ float residual(float r, float mu, float bu0, float bi0, float dot) {
    return (((r - mu) - bu0) - bi0) - dot;
}

// ---------------------------------------------------------------- v0
// Reference kernel: every value read from and written to global memory.
template <int KPL>
__global__ __launch_bounds__(64) void sgd_global_kernel(const Rec *__restrict__ recs,
                                                        const int64_t *__restrict__ block_ptr, int b, int s,
                                                        int64_t rb, int64_t cb, int ibits, int k, float *P, float *Q,
                                                        float *bu, float *bi, float mu, HP hp) {
    const int j = blockIdx.x;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * b + j;
    const int64_t beg = block_ptr[blk], end = block_ptr[blk + 1];
    const uint32_t imask = (1u << ibits) - 1u;
    const int lane = threadIdx.x;
    for (int64_t t = beg; t < end; ++t) {
        const Rec rec = recs[t];
        const int64_t u = (int64_t)br * rb + (rec.ui >> ibits);
        const int64_t i = (int64_t)j * cb + (rec.ui & imask);
        float p[KPL], q[KPL];
#pragma unroll
        for (int c = 0; c < KPL; ++c) {
            const int f = lane + WAVE * c;
            p[c] = f < k ? P[u * k + f] : 0.f;
            q[c] = f < k ? Q[i * k + f] : 0.f;
        }
        const float dot = wave_sum_xor(lane_dot(p, q));
        const float bu0 = bu[u], bi0 = bi[i];
        const float e = residual(rec.r, mu, bu0, bi0, dot);
        factor_update(p, q, e, hp);
#pragma unroll
        for (int c = 0; c < KPL; ++c) {
            const int f = lane + WAVE * c;
            if (f < k) {
                P[u * k + f] = p[c];
                Q[i * k + f] = q[c];
            }
        }
        if (lane == 0) {
            bu[u] = bias_update(bu0, e, hp.a_bu, hp.b_bu);
            bi[i] = bias_update(bi0, e, hp.a_bi, hp.b_bi);
        }
    }
}

// ---------------------------------------------------------------- v1
// LDS-staged kernel.  Workgroup = 4 waves.
//  * The block column's item slice Q[i0 : i0+cb] and bi slice live in LDS
//    for the whole block (read once, written back once).
//  * Ratings go in chunks of 64.  While wave 0 runs the SGD chain over
//    chunk c, waves 1-3 stage chunk c+1: its 64 records and, for every
//    record that starts a new user run, that user's P row and bu into a
//    double buffer.  One barrier per chunk.
//  * Wave 0 keeps the current user's p and bu in registers for the whole
//    run (a user's ratings are contiguous in (u, i) order) and writes them
//    to global memory when the run ends.  A run that crosses a chunk
//    boundary keeps its registers (the staged copy is stale then).
//  * The next rating's item row and bias are read from LDS one rating ahead;
//    when the next rating hits the same item (a duplicate pair) the freshly
//    updated registers are forwarded instead.
constexpr int LDS_WG = 256;
constexpr int CHUNK = 64;

struct LdsLayout {
    int k, ncols;
    size_t q_off, bi_off, rec_off, p_off, bu_off, total;
};

__host__ __device__ inline LdsLayout lds_layout(int k, int64_t cb) {
    LdsLayout L;
    L.k = k;
    L.ncols = (int)cb;
    size_t o = 0;
    L.q_off = o;
    o += (size_t)cb * k * 4;
    L.bi_off = o;
    o += (size_t)cb * 4;
    o = (o + 15) & ~size_t(15);
    L.rec_off = o;
    o += 2 * CHUNK * sizeof(Rec);
    L.p_off = o;
    o += (size_t)2 * CHUNK * k * 4;
    L.bu_off = o;
    o += 2 * CHUNK * 4;
    L.total = o;
    return L;
}

template <int KPL>
__global__ __launch_bounds__(LDS_WG) void sgd_lds_kernel(const Rec *__restrict__ recs,
                                                         const int64_t *__restrict__ block_ptr, int b, int s,
                                                         int64_t n, int64_t rb, int64_t cb, int ibits, int k,
                                                         float *P, float *Q, float *bu, float *bi, float mu,
                                                         HP hp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsLayout L = lds_layout(k, cb);
    float *Qs = reinterpret_cast<float *>(smem + L.q_off);
    float *bis = reinterpret_cast<float *>(smem + L.bi_off);
    Rec *rbuf = reinterpret_cast<Rec *>(smem + L.rec_off);
    float *Ps = reinterpret_cast<float *>(smem + L.p_off);
    float *bus = reinterpret_cast<float *>(smem + L.bu_off);

    const int j = blockIdx.x;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * b + j;
    const int64_t beg = block_ptr[blk], end = block_ptr[blk + 1];
    if (beg == end) return;
    const int64_t i0 = (int64_t)j * cb;
    const int64_t u0 = (int64_t)br * rb;
    const int ncols = (int)std::min<int64_t>(cb, n - i0);
    const uint32_t imask = (1u << ibits) - 1u;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE;
    const int64_t cnt = end - beg;
    const int nchunks = (int)((cnt + CHUNK - 1) / CHUNK);

    // stage the item slice
    for (int64_t x = tid; x < (int64_t)ncols * k; x += LDS_WG) Qs[x] = Q[i0 * k + x];
    for (int x = tid; x < ncols; x += LDS_WG) bis[x] = bi[i0 + x];

    // helpers (waves 1..3): stage chunk c into buffer c & 1
    auto stage = [&](int c) {
        const int buf = c & 1;
        const int64_t cbeg = beg + (int64_t)c * CHUNK;
        const int len = (int)std::min<int64_t>(CHUNK, end - cbeg);
        for (int l = wave - 1; l < len; l += LDS_WG / WAVE - 1) {
            const Rec rec = recs[cbeg + l];
            const uint32_t ul = rec.ui >> ibits;
            const bool start = (l == 0) || (recs[cbeg + l - 1].ui >> ibits) != ul;
            if (lane == 0) {
                rbuf[buf * CHUNK + l] = rec;
                bus[buf * CHUNK + l] = bu[u0 + ul];
            }
            if (start)
                for (int f = lane; f < k; f += WAVE) Ps[((size_t)buf * CHUNK + l) * k + f] = P[(u0 + ul) * k + f];
        }
    };
    if (wave > 0) stage(0);
    __syncthreads();

    float p[KPL], q[KPL], qn[KPL];
    float bu_cur = 0.f;
    int64_t cur_u = -1;  // global id of the user whose p/bu sit in registers

    for (int c = 0; c < nchunks; ++c) {
        if (wave > 0) {
            if (c + 1 < nchunks) stage(c + 1);
        } else {
            const int buf = c & 1;
            const int64_t cbeg = beg + (int64_t)c * CHUNK;
            const int len = (int)std::min<int64_t>(CHUNK, end - cbeg);
            // lane l holds record l of the chunk
            Rec myrec = rbuf[buf * CHUNK + (lane < len ? lane : 0)];
            uint32_t rec_ui = myrec.ui;
            float rec_r = myrec.r;
            // prefetch the first rating's item row
            uint32_t ui_n = __builtin_amdgcn_readlane(rec_ui, 0);
            uint32_t il_n = ui_n & imask;
#pragma unroll
            for (int cc = 0; cc < KPL; ++cc) {
                const int f = lane + WAVE * cc;
                qn[cc] = f < k ? Qs[il_n * k + f] : 0.f;
            }
            float bin = bis[il_n];
            for (int l = 0; l < len; ++l) {
                const uint32_t ui = ui_n;
                const uint32_t il = il_n;
                const float r = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rec_r), l));
                const int64_t u = u0 + (ui >> ibits);
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) q[cc] = qn[cc];
                const float bi0 = bin;
                if (u != cur_u) {
                    if (cur_u >= 0) {
#pragma unroll
                        for (int cc = 0; cc < KPL; ++cc) {
                            const int f = lane + WAVE * cc;
                            if (f < k) P[cur_u * k + f] = p[cc];
                        }
                        if (lane == 0) bu[cur_u] = bu_cur;
                    }
#pragma unroll
                    for (int cc = 0; cc < KPL; ++cc) {
                        const int f = lane + WAVE * cc;
                        p[cc] = f < k ? Ps[((size_t)buf * CHUNK + l) * k + f] : 0.f;
                    }
                    bu_cur = bus[buf * CHUNK + l];
                    cur_u = u;
                }
                // prefetch the next rating's item row (forwarded below when
                // it is the same item)
                const bool has_next = l + 1 < len;
                if (has_next) {
                    ui_n = __builtin_amdgcn_readlane(rec_ui, l + 1);
                    il_n = ui_n & imask;
#pragma unroll
                    for (int cc = 0; cc < KPL; ++cc) {
                        const int f = lane + WAVE * cc;
                        qn[cc] = f < k ? Qs[il_n * k + f] : 0.f;
                    }
                    bin = bis[il_n];
                }
                const float dot = wave_sum_dpp(lane_dot(p, q));
                const float e = residual(r, mu, bu_cur, bi0, dot);
                factor_update(p, q, e, hp);
                const float bi1 = bias_update(bi0, e, hp.a_bi, hp.b_bi);
                bu_cur = bias_update(bu_cur, e, hp.a_bu, hp.b_bu);
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    if (f < k) Qs[il * k + f] = q[cc];
                }
                if (lane == 0) bis[il] = bi1;
                if (has_next && il_n == il) {
#pragma unroll
                    for (int cc = 0; cc < KPL; ++cc) qn[cc] = q[cc];
                    bin = bi1;
                }
            }
        }
        __syncthreads();
    }
    if (wave == 0 && cur_u >= 0) {
#pragma unroll
        for (int cc = 0; cc < KPL; ++cc) {
            const int f = lane + WAVE * cc;
            if (f < k) P[cur_u * k + f] = p[cc];
        }
        if (lane == 0) bu[cur_u] = bu_cur;
    }
    __syncthreads();
    for (int64_t x = tid; x < (int64_t)ncols * k; x += LDS_WG) Q[i0 * k + x] = Qs[x];
    for (int x = tid; x < ncols; x += LDS_WG) bi[i0 + x] = bis[x];
}

// ---------------------------------------------------------------- host
template <int KPL>
static void launch_stratum(Model &M, int s, const HP &hp, int variant, size_t lds_bytes) {
    const Partition &Pt = M.part;
    const float mu = (float)M.mu;
    if (variant == 2) {
        sgd_lds_kernel<KPL><<<M.b, LDS_WG, lds_bytes, M.stream>>>(
            Pt.recs.as<Rec>(), Pt.block_ptr.as<int64_t>(), M.b, s, M.n, Pt.rb, Pt.cb, Pt.ibits, M.k, M.P.as<float>(),
            M.Q.as<float>(), M.bu.as<float>(), M.bi.as<float>(), mu, hp);
    } else {
        sgd_global_kernel<KPL><<<M.b, 64, 0, M.stream>>>(Pt.recs.as<Rec>(), Pt.block_ptr.as<int64_t>(), M.b, s,
                                                          Pt.rb, Pt.cb, Pt.ibits, M.k, M.P.as<float>(),
                                                          M.Q.as<float>(), M.bu.as<float>(), M.bi.as<float>(), mu,
                                                          hp);
    }
    BMF_HIP(hipGetLastError());
}

template <int KPL>
static void set_lds_attr(size_t bytes) {
    static size_t done = 0;
    if (bytes > done) {
        BMF_HIP(hipFuncSetAttribute((const void *)sgd_lds_kernel<KPL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)bytes));
        done = bytes;
    }
}

static int max_lds_bytes(int device) {
    static int cached[64] = {0};
    if (device < 64 && cached[device]) return cached[device];
    int v = 0;
    BMF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (device < 64) cached[device] = v;
    return v;
}

void sgd_epoch(Model &M, const int32_t *order, const HP &hp) {
    const int kpl = (M.k + WAVE - 1) / WAVE;
    const LdsLayout L = lds_layout(M.k, M.part.cb);
    int variant = M.sgd_kernel;
    if (variant == 0) variant = ((int64_t)L.total <= max_lds_bytes(M.device)) ? 2 : 1;
    if (variant == 2 && (int64_t)L.total > max_lds_bytes(M.device))
        BMF_FAIL(BMF_E_STATE, "item slice does not fit in LDS for this block grid; use SGD kernel 1 or a larger b");
    if (variant == 2) {
        switch (kpl) {
        case 1: set_lds_attr<1>(L.total); break;
        case 2: set_lds_attr<2>(L.total); break;
        case 3: set_lds_attr<3>(L.total); break;
        case 4: set_lds_attr<4>(L.total); break;
        default: break;
        }
    }
    hipEvent_t ev0 = take_event(M), ev1 = take_event(M);
    BMF_HIP(hipEventRecord(ev0, M.stream));
    for (int pos = 0; pos < M.b; ++pos) {
        const int s = order[pos];
        switch (kpl) {
        case 1: launch_stratum<1>(M, s, hp, variant, L.total); break;
        case 2: launch_stratum<2>(M, s, hp, variant, L.total); break;
        case 3: launch_stratum<3>(M, s, hp, variant, L.total); break;
        case 4: launch_stratum<4>(M, s, hp, variant, L.total); break;
        case 5: launch_stratum<5>(M, s, hp, 1, 0); break;
        case 6: launch_stratum<6>(M, s, hp, 1, 0); break;
        case 7: launch_stratum<7>(M, s, hp, 1, 0); break;
        case 8: launch_stratum<8>(M, s, hp, 1, 0); break;
        default: launch_stratum<16>(M, s, hp, 1, 0); break;
        }
    }
    BMF_HIP(hipEventRecord(ev1, M.stream));
    M.pending.emplace_back(ev0, ev1);
    M.sgd_launches += M.b;
    if (M.pending.size() > 64) harvest_timing(M, false);
}

hipEvent_t take_event(Model &M) {
    if (!M.spare_events.empty()) {
        hipEvent_t e = M.spare_events.back();
        M.spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    BMF_HIP(hipEventCreate(&e));
    return e;
}

void harvest_timing(Model &M, bool wait) {
    size_t done = 0;
    for (; done < M.pending.size(); ++done) {
        auto &pr = M.pending[done];
        if (wait) {
            BMF_HIP(hipEventSynchronize(pr.second));
        } else if (hipEventQuery(pr.second) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        float ms = 0.f;
        BMF_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        M.sgd_ms += ms;
        M.spare_events.push_back(pr.first);
        M.spare_events.push_back(pr.second);
    }
    M.pending.erase(M.pending.begin(), M.pending.begin() + done);
}

// ------------------------------------------------------------ diagnostics
__global__ void debug_wave_sum_kernel(const float *in, float *out) {
    const int lane = threadIdx.x;
    const float v = in[lane];
    const float a = wave_sum_xor(v);
    const float b = wave_sum_dpp(v);
    const float c = row16_sum(v);
    out[lane] = a;
    out[64 + lane] = b;
    out[128 + lane] = c;
}

void debug_wave_sum(const float *d_in, float *d_out, hipStream_t s) {
    debug_wave_sum_kernel<<<1, 64, 0, s>>>(d_in, d_out);
    BMF_HIP(hipGetLastError());
}

}  // namespace bmf
