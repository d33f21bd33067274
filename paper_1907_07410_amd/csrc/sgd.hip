// Stratified block SGD (Algorithm 1's epoch loop with Algorithm 2 as the
// per-block kernel; Eqs 10-13 as the per-rating update).
//
// One stratum s = {((j + s) mod b, j) : j < b} is one launch: workgroup j
// owns block ((j + s) mod b, j).  Blocks of a stratum share no block row and
// no block column (Section 3, parallel BMF), so the workgroups touch
// disjoint rows of P/bu and of Q/bi; the stream order between launches is
// the barrier between strata.
//
// Inside a block the ratings are updated in (u, i, t) order (Algorithm 2),
// or in a plan's steps, which reorder only ratings that share neither user
// nor item and so give the same bits.  For k <= 128 a rating is handled by
// 16 lanes (lane l owns factors l*F .. l*F + F - 1, F = 1, 2, 4 or 8) and
// both kernels that use this layout perform the same floating-point
// operations in the same order (the helpers below): the reference kernel
// (global memory, processing order) and the planned LDS kernel agree bit for
// bit.  For k > 128 the reference kernel spreads a rating over all 64 lanes
// (lane f owns factors f, f + 64, ...).
#pragma clang fp contract(off)

#include <algorithm>
#include <cstring>

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

// Eqs 10 and 11 from pre-update values:
//   self + alpha (err * other - beta * self)
//     = fma(alpha * err, other, fma(-(alpha * beta), self, self)),
// two FMAs per factor with the products alpha*err (per rating) and
// alpha*beta (a constant) rounded once.  The decay self - alpha beta self is
// one rounding of the exact value, so no rounding is repeated the same way
// at every update.  Every kernel uses this helper and rounds identically.
template <int KPL>
__device__ __forceinline__ void factor_update(float (&p)[KPL], float (&q)[KPL], float e, const HP &hp) {
    const float ape = hp.a_p * e, aqe = hp.a_q * e;
    const float dp = -(hp.a_p * hp.b_p), dq = -(hp.a_q * hp.b_q);
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
        const float pc = p[c], qc = q[c];
        p[c] = fmaf(ape, qc, fmaf(dp, pc, pc));
        q[c] = fmaf(aqe, pc, fmaf(dq, qc, qc));
    }
}

__device__ __forceinline__ float bias_update(float b0, float e, float a, float beta) {
    return fmaf(a, fmaf(-beta, b0, e), b0);
}

__device__ __forceinline__ float residual(float r, float mu, float bu0, float bi0, float dot) {
    return (((r - mu) - bu0) - bi0) - dot;
}

// ---------------------------------------------------------- v0, k > 128
// Reference kernel for k > 128: every value read from and written to global
// memory, one wavefront per block.
template <int KPL>
__global__ __launch_bounds__(64) void sgd_global_kernel(const Rec *__restrict__ recs,
                                                        const int64_t *__restrict__ block_ptr, int b, int s,
                                                        int64_t row_stride, int64_t rb, int64_t cb, int ibits, int k,
                                                        float *P, float *Q, float *bu, float *bi, float mu, HP hp) {
    const int j = blockIdx.x;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * row_stride + j;
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

// ------------------------------------------------------------ v0, k <= 128
// Reference kernel in the 16-lane layout the planned kernel uses: one
// 16-lane row per block (a workgroup of 64 threads runs four blocks of the
// stratum), lane l owns factors l*F .. l*F + F - 1, everything in global
// memory, ratings in processing order.  Its arithmetic is the planned
// kernel's, so the two agree bit for bit.
template <int F>
__global__ __launch_bounds__(64) void sgd_ref16_kernel(const Rec *__restrict__ recs,
                                                       const int64_t *__restrict__ block_ptr, int b, int s,
                                                       int64_t row_stride, int64_t rb, int64_t cb, int ibits, int k,
                                                       float *P, float *Q, float *bu, float *bi, float mu, HP hp) {
    const int row = threadIdx.x >> 4, gl = threadIdx.x & 15;
    const int j = blockIdx.x * 4 + row;
    if (j >= b) return;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * row_stride + j;
    const int64_t beg = block_ptr[blk], end = block_ptr[blk + 1];
    const uint32_t imask = (1u << ibits) - 1u;
    for (int64_t t = beg; t < end; ++t) {
        const Rec rec = recs[t];
        const int64_t u = (int64_t)br * rb + (rec.ui >> ibits);
        const int64_t i = (int64_t)j * cb + (rec.ui & imask);
        float p[F], q[F];
#pragma unroll
        for (int c = 0; c < F; ++c) {
            const int f = gl * F + c;
            p[c] = f < k ? P[u * k + f] : 0.f;
            q[c] = f < k ? Q[i * k + f] : 0.f;
        }
        const float dot = row16_sum(lane_dot(p, q));
        const float bu0 = bu[u], bi0 = bi[i];
        const float e = residual(rec.r, mu, bu0, bi0, dot);
        factor_update(p, q, e, hp);
#pragma unroll
        for (int c = 0; c < F; ++c) {
            const int f = gl * F + c;
            if (f < k) {
                P[u * k + f] = p[c];
                Q[i * k + f] = q[c];
            }
        }
        if (gl == 0) {
            bu[u] = bias_update(bu0, e, hp.a_bu, hp.b_bu);
            bi[i] = bias_update(bi0, e, hp.a_bi, hp.b_bi);
        }
    }
}

// ---------------------------------------------------------------- v1
// Planned LDS kernel.  A block's ratings run in the steps of its plan
// (plan.hip): four mutually independent ratings per step, one per 16-lane
// group of wavefront 0, which touches only LDS:
//  * the block column's item slice (Q rows and bi) is staged once and
//    written back once;
//  * every user active in the block has an LDS slot holding p_u and bu_u;
//  * per step each group reads its slot record (item, slot, rating), its
//    user and item rows, does the update of Eqs 10-13 with the dot product
//    summed over its 16 lanes, and writes both rows back.  Records carry
//    the rows' LDS addresses, and each row keeps its bias after the
//    factors.  Empty positions point at a dummy user slot and a dummy item
//    row.
// The other wavefronts are helpers.  Steps go in chunks of CH; while
// wavefront 0 runs chunk c the helpers write back to global memory the user
// rows whose last rating was in chunk c-1 and stage chunk c+1: its slot
// records and the rows of users whose first rating is in it.  The plan
// keeps a slot idle for two chunks between its users, so these never touch
// a slot wavefront 0 is using.  One barrier per chunk; records are triple
// buffered (chunk c-1 read by the write-back, c by the chain, c+1 staged).
template <int F>
__device__ __forceinline__ void row_ld(float (&v)[F], const float *a) {
    if constexpr (F == 1) {
        v[0] = a[0];
    } else if constexpr (F == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(a);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int c = 0; c < F; c += 4) {
            const float4 t = *reinterpret_cast<const float4 *>(a + c);
            v[c] = t.x;
            v[c + 1] = t.y;
            v[c + 2] = t.z;
            v[c + 3] = t.w;
        }
    }
}

template <int F>
__device__ __forceinline__ void row_st(float *a, const float (&v)[F]) {
    if constexpr (F == 1) {
        a[0] = v[0];
    } else if constexpr (F == 2) {
        *reinterpret_cast<float2 *>(a) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int c = 0; c < F; c += 4) *reinterpret_cast<float4 *>(a + c) = make_float4(v[c], v[c + 1], v[c + 2], v[c + 3]);
    }
}

// One step of the chain wavefront: lane group g (16 lanes) takes its record
// rec = {item row LDS offset, rating bits, user slot LDS offset, -}, reads
// both rows and biases from LDS, sums the dot product over its 16 lanes,
// applies Eqs 10-13 and writes the rows back.
template <int F>
__device__ __forceinline__ void plan_step(unsigned char *smem, const uint4 rec, int gl, float mu, const HP &hp) {
    constexpr int KP = 16 * F;
    float *urow = reinterpret_cast<float *>(smem + rec.z);
    float *qrow = reinterpret_cast<float *>(smem + rec.x);
    const float bu0 = urow[KP], bi0 = qrow[KP];
    float p[F], q[F];
    row_ld<F>(p, urow + gl * F);
    row_ld<F>(q, qrow + gl * F);
    const float dot = row16_sum(lane_dot(p, q));
    const float e = residual(__uint_as_float(rec.y), mu, bu0, bi0, dot);
    factor_update(p, q, e, hp);
    row_st<F>(urow + gl * F, p);
    row_st<F>(qrow + gl * F, q);
    urow[KP] = bias_update(bu0, e, hp.a_bu, hp.b_bu);
    qrow[KP] = bias_update(bi0, e, hp.a_bi, hp.b_bi);
}

// The chain wavefront's loop over one chunk of len steps (records rb, four
// per step): steps in groups of four (then two, one), so the registers a
// step writes back from are not the ones the next step loads into.
template <int F>
__device__ __forceinline__ void plan_chunk(unsigned char *smem, const SlotRec *rb, int len, int g, int gl, float mu,
                                           const HP &hp) {
    int t = 0;
    for (; t + 3 < len; t += 4) {
        const uint4 r0 = *reinterpret_cast<const uint4 *>(&rb[t * PLAN_W + g]);
        const uint4 r1 = *reinterpret_cast<const uint4 *>(&rb[(t + 1) * PLAN_W + g]);
        const uint4 r2 = *reinterpret_cast<const uint4 *>(&rb[(t + 2) * PLAN_W + g]);
        const uint4 r3 = *reinterpret_cast<const uint4 *>(&rb[(t + 3) * PLAN_W + g]);
        plan_step<F>(smem, r0, gl, mu, hp);
        plan_step<F>(smem, r1, gl, mu, hp);
        plan_step<F>(smem, r2, gl, mu, hp);
        plan_step<F>(smem, r3, gl, mu, hp);
    }
    for (; t + 1 < len; t += 2) {
        const uint4 r0 = *reinterpret_cast<const uint4 *>(&rb[t * PLAN_W + g]);
        const uint4 r1 = *reinterpret_cast<const uint4 *>(&rb[(t + 1) * PLAN_W + g]);
        plan_step<F>(smem, r0, gl, mu, hp);
        plan_step<F>(smem, r1, gl, mu, hp);
    }
    if (t < len) plan_step<F>(smem, *reinterpret_cast<const uint4 *>(&rb[t * PLAN_W + g]), gl, mu, hp);
}

__device__ __forceinline__ int lane_rank(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int F, bool VEC, int NW>
__device__ __forceinline__ void planned_block(const SlotRec *__restrict__ steps, int64_t nsteps, int64_t u0,
                                              int64_t i0, int64_t n, int64_t cb, int k, int S, int CH, float *P,
                                              float *Q, float *bu, float *bi, float mu, const HP &hp,
                                              unsigned char *smem) {
    constexpr int KP = 16 * F;
    constexpr int RS = KP + 4;  // floats per LDS row: factors, bias, padding
    constexpr int WG = NW * WAVE;
    constexpr int NH = NW - 1;
    constexpr int RB = 2;  // rows in flight per 16-lane group while staging
    if (nsteps <= 0) return;
    const PlanLds L = plan_lds(KP, cb, S, CH);
    float *Qs = reinterpret_cast<float *>(smem + L.q);
    SlotRec *Rb = reinterpret_cast<SlotRec *>(smem + L.rec);
    uint2 *Scr = reinterpret_cast<uint2 *>(smem + L.scr);
    float *Us = reinterpret_cast<float *>(smem + L.u);
    const int ncols = (int)std::min<int64_t>(cb, n - i0);
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE;
    const int g = lane >> 4, gl = lane & 15;
    const int RPC = CH * PLAN_W;
    const int nch = (int)((nsteps + CH - 1) / CH);

    // item slice: factors (zero beyond k) and bias per row; dummy item row
    // and dummy user slot zeroed
    for (int64_t x = tid; x < (int64_t)ncols * KP; x += WG) {
        const int64_t il = x / KP;
        const int f = (int)(x % KP);
        Qs[il * RS + f] = f < k ? Q[(i0 + il) * k + f] : 0.f;
    }
    for (int x = tid; x < ncols; x += WG) Qs[(int64_t)x * RS + KP] = bi[i0 + x];
    if (tid < RS) {
        Qs[(size_t)cb * RS + tid] = 0.f;
        Us[(size_t)S * RS + tid] = 0.f;
    }

    const int hw = wave - 1;
    uint2 *scr = Scr + (size_t)(hw < 0 ? 0 : hw) * WAVE;

    // helpers: write back the users whose last rating is in chunk c
    auto write_back = [&](int c) {
        const int cnt = (int)std::min<int64_t>(CH, nsteps - (int64_t)c * CH) * PLAN_W;
        const SlotRec *src = Rb + (size_t)(c % 3) * RPC;
        for (int base = 0; base < cnt; base += NH * WAVE) {
            const int x = base + lane * NH + hw;
            const bool valid = x < cnt;
            SlotRec rec{0u, 0.f, 0u, 0u};
            if (valid) rec = src[x];
            const bool last = valid && (rec.ulf & PLAN_LAST);
            const uint64_t mask = __ballot(last);
            const int nl = __popcll(mask);
            if (last) scr[lane_rank(mask)] = make_uint2(rec.ulf & PLAN_UL_MASK, rec.ua);
            for (int e = g; e < nl; e += 4) {
                const uint2 en = scr[e];
                const int64_t row = u0 + en.x;
                const float *srow = reinterpret_cast<const float *>(smem + en.y);
                float v[F];
                row_ld<F>(v, srow + gl * F);
                if (VEC) {
                    row_st<F>(P + row * k + gl * F, v);
                } else {
#pragma unroll
                    for (int c2 = 0; c2 < F; ++c2)
                        if (gl * F + c2 < k) P[row * k + gl * F + c2] = v[c2];
                }
                if (gl == 0) bu[row] = srow[KP];
            }
        }
    };
    // helpers: stage chunk c (records, and the rows of users starting in it)
    auto stage = [&](int c) {
        const int64_t s0 = (int64_t)c * CH;
        const int cnt = (int)std::min<int64_t>(CH, nsteps - s0) * PLAN_W;
        SlotRec *dst = Rb + (size_t)(c % 3) * RPC;
        const SlotRec *src = steps + s0 * PLAN_W;
        for (int base = 0; base < cnt; base += NH * WAVE) {
            const int x = base + lane * NH + hw;
            const bool valid = x < cnt;
            SlotRec rec{0u, 0.f, 0u, 0u};
            if (valid) rec = src[x];
            const bool first = valid && (rec.ulf & PLAN_FIRST);
            if (valid) dst[x] = rec;
            const uint64_t mask = __ballot(first);
            const int nf = __popcll(mask);
            if (first) scr[lane_rank(mask)] = make_uint2(rec.ulf & PLAN_UL_MASK, rec.ua);
            for (int e0 = 0; e0 < nf; e0 += 4 * RB) {
                float v[RB][F];
                float bv[RB];
                uint32_t ua[RB];
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    const int e = e0 + 4 * jj + g;
                    ua[jj] = 0xffffffffu;
                    bv[jj] = 0.f;
#pragma unroll
                    for (int c2 = 0; c2 < F; ++c2) v[jj][c2] = 0.f;
                    if (e < nf) {
                        const uint2 en = scr[e];
                        ua[jj] = en.y;
                        const int64_t row = u0 + en.x;
                        if (VEC) {
                            row_ld<F>(v[jj], P + row * k + gl * F);
                        } else {
#pragma unroll
                            for (int c2 = 0; c2 < F; ++c2)
                                if (gl * F + c2 < k) v[jj][c2] = P[row * k + gl * F + c2];
                        }
                        bv[jj] = bu[row];
                    }
                }
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    if (ua[jj] != 0xffffffffu) {
                        float *drow = reinterpret_cast<float *>(smem + ua[jj]);
                        row_st<F>(drow + gl * F, v[jj]);
                        drow[KP] = bv[jj];
                    }
                }
            }
        }
    };

    if (wave > 0) stage(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (wave == 0) {
            const int len = (int)std::min<int64_t>(CH, nsteps - (int64_t)c * CH);
            plan_chunk<F>(smem, Rb + (size_t)(c % 3) * RPC, len, g, gl, mu, hp);
        } else {
            if (c > 0) write_back(c - 1);
            if (c + 1 < nch) stage(c + 1);
        }
        __syncthreads();
    }
    if (wave > 0) write_back(nch - 1);
    __syncthreads();
    for (int64_t x = tid; x < (int64_t)ncols * KP; x += WG) {
        const int64_t il = x / KP;
        const int f = (int)(x % KP);
        if (f < k) Q[(i0 + il) * k + f] = Qs[il * RS + f];
    }
    for (int x = tid; x < ncols; x += WG) bi[i0 + x] = Qs[(int64_t)x * RS + KP];
}

// One stratum s: workgroup j owns block ((j + s) mod b, j).  Block tables
// (here and in the reference kernels) are indexed br * row_stride + j:
// row_stride b for tables over the whole grid, 0 for a table of the
// stratum's own blocks in position order.
template <int F, bool VEC, int NW>
__global__ __launch_bounds__(NW *WAVE) void sgd_plan_kernel(const SlotRec *__restrict__ steps,
                                                            const int64_t *__restrict__ blk_step, int b, int s,
                                                            int64_t row_stride, int64_t n, int64_t rb, int64_t cb,
                                                            int k, int S, int CH, float *P, float *Q, float *bu,
                                                            float *bi, float mu, HP hp) {
    __shared__ __align__(16) unsigned char smem[PLAN_LDS_BYTES];
    const int j = blockIdx.x;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * row_stride + j;
    const int64_t s0 = blk_step[blk];
    planned_block<F, VEC, NW>(steps + s0 * PLAN_W, blk_step[blk + 1] - s0, (int64_t)br * rb, (int64_t)j * cb, n, cb,
                              k, S, CH, P, Q, bu, bi, mu, hp, smem);
}

// ------------------------------------------------------------- batched
// Many independent problems trained together.  Global position t of problem
// p is epoch t / b_p, position t % b_p of that epoch's stratum order; one
// launch runs position t of every problem that has one: workgroup g takes
// item items[first + g] = (problem, t, stratum s, column j) and runs block
// ((j + s) mod b_p, j) of that problem.  Blocks of one position of one
// problem form a stratum (no shared row or column); blocks of different
// problems share nothing; successive positions are ordered by the stream.
template <int F, bool VEC, int NW>
__global__ __launch_bounds__(NW *WAVE) void sgd_positions_kernel(const BatchProblem *__restrict__ probs,
                                                                 const BatchItem *__restrict__ items, int k,
                                                                 HP hp) {
    __shared__ __align__(16) unsigned char smem[PLAN_LDS_BYTES];
    const BatchItem it = items[blockIdx.x];
    const BatchProblem pr = probs[it.p];
    const int r = (it.j + it.s) % pr.b;
    const int64_t blk = (int64_t)r * pr.b + it.j;
    const int64_t s0 = pr.blk_step[blk];
    planned_block<F, VEC, NW>(pr.steps + s0 * PLAN_W, pr.blk_step[blk + 1] - s0, (int64_t)r * pr.rb,
                              (int64_t)it.j * pr.cb, pr.n, pr.cb, k, pr.S, pr.CH, pr.P, pr.Q, pr.bu, pr.bi, pr.mu,
                              hp, smem);
}

// ---------------------------------------------------------------- host
template <int KPL>
static void launch_global(Model &M, int s, const HP &hp, const StratumData &D) {
    const Partition &Pt = M.part;
    sgd_global_kernel<KPL><<<M.b, 64, 0, M.stream>>>(static_cast<const Rec *>(D.data), D.table, M.b, s, D.row_stride,
                                                      Pt.rb, Pt.cb, Pt.ibits, M.k, M.P.as<float>(), M.Q.as<float>(),
                                                      M.bu.as<float>(), M.bi.as<float>(), (float)M.mu, hp);
    BMF_HIP(hipGetLastError());
}

template <int F>
static void launch_ref16(Model &M, int s, const HP &hp, const StratumData &D) {
    const Partition &Pt = M.part;
    sgd_ref16_kernel<F><<<(M.b + 3) / 4, 64, 0, M.stream>>>(static_cast<const Rec *>(D.data), D.table, M.b, s,
                                                           D.row_stride, Pt.rb, Pt.cb, Pt.ibits, M.k,
                                                           M.P.as<float>(), M.Q.as<float>(), M.bu.as<float>(),
                                                           M.bi.as<float>(), (float)M.mu, hp);
    BMF_HIP(hipGetLastError());
}

template <int F, bool VEC, int NW>
static void launch_plan(Model &M, int s, const HP &hp, const StratumData &D) {
    sgd_plan_kernel<F, VEC, NW><<<M.b, NW * WAVE, 0, M.stream>>>(
        static_cast<const SlotRec *>(D.data), D.table, M.b, s, D.row_stride, M.n, M.part.rb, M.part.cb, M.k,
        M.plan.S, M.plan.CH, M.P.as<float>(), M.Q.as<float>(), M.bu.as<float>(), M.bi.as<float>(), (float)M.mu, hp);
    BMF_HIP(hipGetLastError());
}

int sgd_max_lds(int device) {
    static int cached[64] = {0};
    if (device < 64 && cached[device]) return cached[device];
    int v = 0;
    BMF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (device < 64) cached[device] = v;
    return v;
}

// dispatch key of the planned kernels: F in {1, 2, 4, 8}, k == 16 F, waves
static int plan_key(int k, int nw) {
    const int kp = plan_kp(k);
    const int fi = kp == 16 ? 0 : kp == 32 ? 1 : kp == 64 ? 2 : 3;
    return fi * 4 + (k == kp ? 2 : 0) + (nw == 8 ? 1 : 0);
}

void launch_stratum(Model &M, int s, const HP &hp, int variant, const StratumData &D) {
    if (variant == 2) {
        switch (plan_key(M.k, M.waves)) {
        case 0: launch_plan<1, false, 4>(M, s, hp, D); return;
        case 1: launch_plan<1, false, 8>(M, s, hp, D); return;
        case 2: launch_plan<1, true, 4>(M, s, hp, D); return;
        case 3: launch_plan<1, true, 8>(M, s, hp, D); return;
        case 4: launch_plan<2, false, 4>(M, s, hp, D); return;
        case 5: launch_plan<2, false, 8>(M, s, hp, D); return;
        case 6: launch_plan<2, true, 4>(M, s, hp, D); return;
        case 7: launch_plan<2, true, 8>(M, s, hp, D); return;
        case 8: launch_plan<4, false, 4>(M, s, hp, D); return;
        case 9: launch_plan<4, false, 8>(M, s, hp, D); return;
        case 10: launch_plan<4, true, 4>(M, s, hp, D); return;
        case 11: launch_plan<4, true, 8>(M, s, hp, D); return;
        case 12: launch_plan<8, false, 4>(M, s, hp, D); return;
        case 13: launch_plan<8, false, 8>(M, s, hp, D); return;
        case 14: launch_plan<8, true, 4>(M, s, hp, D); return;
        default: launch_plan<8, true, 8>(M, s, hp, D); return;
        }
    }
    switch (plan_kp(M.k)) {
    case 16: launch_ref16<1>(M, s, hp, D); return;
    case 32: launch_ref16<2>(M, s, hp, D); return;
    case 64: launch_ref16<4>(M, s, hp, D); return;
    case 128: launch_ref16<8>(M, s, hp, D); return;
    default: break;
    }
    switch ((M.k + WAVE - 1) / WAVE) {
    case 3: launch_global<3>(M, s, hp, D); break;
    case 4: launch_global<4>(M, s, hp, D); break;
    case 5: launch_global<5>(M, s, hp, D); break;
    case 6: launch_global<6>(M, s, hp, D); break;
    case 7: launch_global<7>(M, s, hp, D); break;
    case 8: launch_global<8>(M, s, hp, D); break;
    default: launch_global<16>(M, s, hp, D); break;
    }
}

void ensure_plan(Model &M) {
    if (!M.plan.built) build_plan(M.plan, M.part, M.b, M.k, sgd_max_lds(M.device), M.stream);
}

void EpochGraph::reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
}

// The epoch's launches through the cached graph, captured again whenever
// anything the launches depend on has changed since the last capture.
static void graph_epoch(Model &M, const int32_t *order, const HP &hp, int variant, const StratumData &D) {
    auto bits = [](float x) {
        uint32_t u;
        std::memcpy(&u, &x, 4);
        return (uint64_t)u;
    };
    const float muf = (float)M.mu;
    std::vector<uint64_t> key = {(uint64_t)variant, (uint64_t)M.b, (uint64_t)M.k, (uint64_t)M.n, (uint64_t)M.waves,
                                 (uint64_t)(uintptr_t)D.data, (uint64_t)(uintptr_t)D.table, (uint64_t)D.row_stride,
                                 (uint64_t)(uintptr_t)M.P.p, (uint64_t)(uintptr_t)M.Q.p, (uint64_t)(uintptr_t)M.bu.p,
                                 (uint64_t)(uintptr_t)M.bi.p, (uint64_t)M.part.rb, (uint64_t)M.part.cb,
                                 (uint64_t)M.part.ibits, (uint64_t)M.plan.S, (uint64_t)M.plan.CH, bits(muf),
                                 bits(hp.a_p), bits(hp.b_p), bits(hp.a_q), bits(hp.b_q), bits(hp.a_bu), bits(hp.b_bu),
                                 bits(hp.a_bi), bits(hp.b_bi)};
    for (int pos = 0; pos < M.b; ++pos) key.push_back((uint64_t)(uint32_t)order[pos]);
    EpochGraph &E = M.egraph;
    if (!E.exec || key != E.key) {
        E.reset();
        BMF_HIP(hipStreamBeginCapture(M.stream, hipStreamCaptureModeThreadLocal));
        try {
            for (int pos = 0; pos < M.b; ++pos) launch_stratum(M, order[pos], hp, variant, D);
        } catch (...) {
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(M.stream, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            throw;
        }
        BMF_HIP(hipStreamEndCapture(M.stream, &E.graph));
        BMF_HIP(hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0));
        E.key = std::move(key);
        E.captures += 1;
    }
    BMF_HIP(hipGraphLaunch(E.exec, M.stream));
}

int sgd_variant(Model &M) {
    int variant = M.sgd_kernel;
    if (M.ooc.on) {
        if (variant == 0) variant = M.ooc.variant;
        if (variant != M.ooc.variant)
            BMF_FAIL(BMF_E_STATE, "out-of-core ratings were laid out for SGD kernel " + std::to_string(M.ooc.variant) +
                                      "; set the kernel before loading");
    }
    if (variant == 0) variant = M.plan.ok && plan_pays(M.part.nnz, M.b) ? 2 : 1;
    if (variant == 2) ensure_plan(M);
    if (variant == 2 && !M.plan.ok)
        BMF_FAIL(BMF_E_STATE, "the LDS-staged SGD kernel needs k <= 128 and an item slice that leaves room for "
                              "user slots in LDS; use SGD kernel 1 or a larger b");
    return variant;
}

void sgd_epoch(Model &M, const int32_t *order, const HP &hp) {
    const int variant = sgd_variant(M);
    if (!M.ooc.on && disjoint_check_env()) {
        const int64_t bad = disjoint_check(M, variant, nullptr);
        if (bad)
            BMF_FAIL(BMF_E_STATE, "race check: " + std::to_string(bad) +
                                      " ratings share a row with another block of their stratum");
    }
    hipEvent_t ev0 = take_event(M), ev1 = take_event(M);
    BMF_HIP(hipEventRecord(ev0, M.stream));
    if (M.ooc.on) {
        ooc_epoch(M, order, hp, variant);
    } else {
        const StratumData D = variant == 2 ? StratumData{M.plan.steps.p, M.plan.blk_step.as<int64_t>(), M.b}
                                           : StratumData{M.part.recs.p, M.part.block_ptr.as<int64_t>(), M.b};
        if (M.egraph.on)
            graph_epoch(M, order, hp, variant, D);
        else
            for (int pos = 0; pos < M.b; ++pos) launch_stratum(M, order[pos], hp, variant, D);
    }
    BMF_HIP(hipEventRecord(ev1, M.stream));
    M.pending.emplace_back(ev0, ev1);
    M.sgd_launches += M.b;
    if (M.pending.size() > 64) harvest_timing(M, false);
}

template <int F, bool VEC, int NW>
static void launch_positions(const BatchProblem *d_probs, const BatchItem *d_items, int64_t count, int k,
                             const HP &hp, size_t lds, hipStream_t s) {
    if (lds > (size_t)PLAN_LDS_BYTES) BMF_FAIL(BMF_E_STATE, "plan exceeds the LDS kernel's buffer");
    sgd_positions_kernel<F, VEC, NW><<<(unsigned)count, NW * WAVE, 0, s>>>(d_probs, d_items, k, hp);
    BMF_HIP(hipGetLastError());
}

void sgd_positions_launch(int k, int nw, const BatchProblem *d_probs, const BatchItem *d_items, int64_t count,
                          const HP &hp, size_t lds, hipStream_t s) {
    if (count == 0) return;
    if (!plan_kp(k) || (nw != 4 && nw != 8))
        BMF_FAIL(BMF_E_INVAL, "batched training needs k <= 128 and 4 or 8 waves per block");
    switch (plan_key(k, nw)) {
    case 0: launch_positions<1, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 1: launch_positions<1, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 2: launch_positions<1, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 3: launch_positions<1, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 4: launch_positions<2, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 5: launch_positions<2, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 6: launch_positions<2, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 7: launch_positions<2, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 8: launch_positions<4, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 9: launch_positions<4, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 10: launch_positions<4, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 11: launch_positions<4, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 12: launch_positions<8, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 13: launch_positions<8, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 14: launch_positions<8, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    default: launch_positions<8, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    }
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
// Dependent-step floor of the planned kernel: one wavefront runs the chain
// wavefront's chunk loop (plan_chunk, the same code) over chunks whose four
// records per step always name the same user slot and item row per lane
// group, so every step reads the rows the step before it wrote: a chain of
// dependent steps with no staging, no barrier and no other wavefront.  Rows
// start at small values and out[] receives a row so that nothing is
// optimised away.
template <int F>
__global__ __launch_bounds__(64) void chain_floor_kernel(int chunks, float mu, HP hp, float *out) {
    constexpr int KP = 16 * F, RS = KP + 4;
    __shared__ __align__(16) unsigned char smem[(8 * RS) * 4 + PLAN_CH * PLAN_W * sizeof(SlotRec)];
    float *rows = reinterpret_cast<float *>(smem);
    SlotRec *rb = reinterpret_cast<SlotRec *>(smem + 8 * RS * 4);
    const int lane = threadIdx.x, g = lane >> 4, gl = lane & 15;
    for (int x = lane; x < 8 * RS; x += WAVE) rows[x] = 0.01f * (float)((x % 7) + 1);
    for (int x = lane; x < PLAN_CH * PLAN_W; x += WAVE) {
        const int gg = x % PLAN_W;
        rb[x] = SlotRec{(uint32_t)(gg * RS * 4), 3.0f + 0.5f * (float)gg, (uint32_t)((4 + gg) * RS * 4), 0u};
    }
    __syncthreads();
    for (int c = 0; c < chunks; ++c) plan_chunk<F>(smem, rb, PLAN_CH, g, gl, mu, hp);
    __syncthreads();
    for (int x = lane; x < 8 * RS; x += WAVE) out[x] = rows[x];
}

void chain_floor(int k, int chunks, float *d_out, hipStream_t s) {
    const HP hp{0.005f, 0.05f, 0.005f, 0.05f, 0.005f, 0.05f, 0.005f, 0.05f};
    switch (plan_kp(k)) {
    case 16: chain_floor_kernel<1><<<1, 64, 0, s>>>(chunks, 3.5f, hp, d_out); break;
    case 32: chain_floor_kernel<2><<<1, 64, 0, s>>>(chunks, 3.5f, hp, d_out); break;
    case 64: chain_floor_kernel<4><<<1, 64, 0, s>>>(chunks, 3.5f, hp, d_out); break;
    case 128: chain_floor_kernel<8><<<1, 64, 0, s>>>(chunks, 3.5f, hp, d_out); break;
    default: BMF_FAIL(BMF_E_INVAL, "the planned kernel's step needs k <= 128");
    }
    BMF_HIP(hipGetLastError());
}

__global__ void debug_wave_sum_kernel(const float *in, float *out) {
    const int lane = threadIdx.x;
    const float v = in[lane];
    const float a = wave_sum_xor(v);
    const float b = wave_sum_dpp(v);
    const float c = row16_sum(v);
    const float d = wave_sum_perm(v);
    out[lane] = a;
    out[64 + lane] = b;
    out[128 + lane] = c;
    out[192 + lane] = d;
}

void debug_wave_sum(const float *d_in, float *d_out, hipStream_t s) {
    debug_wave_sum_kernel<<<1, 64, 0, s>>>(d_in, d_out);
    BMF_HIP(hipGetLastError());
}

}  // namespace bmf
