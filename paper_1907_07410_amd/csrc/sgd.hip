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
// same floating-point operations in the same order (the helpers below), so all
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
// LDS-staged kernel.  Workgroup = 4 waves: wave 0 runs the dependent
// update chain, waves 1-3 move data.
//  * The block column's item slice Q[i0 : i0+cb] and bi slice live in LDS
//    for the whole block (read once, written back once).
//  * Ratings go in chunks of 64.  While wave 0 works on chunk c, the helper
//    waves (a) write back to global memory the user rows whose run ended in
//    chunk c-1 and (b) stage chunk c+1: its records and, for every record
//    that starts a user run, that user's P row and bu, into the other half
//    of a double buffer.  One barrier per chunk.
//  * Wave 0 touches no global memory: it keeps the current user's p and bu
//    in registers (a user's ratings are contiguous in (u, i) order), reads
//    the next rating's item row, item bias and (possibly new) user row from
//    LDS one rating ahead, and after every rating writes the updated item
//    row and bias back to the slice and the updated user row and bias to
//    the rating's staging slot, where the helpers find the final values of
//    each run.  The loop body has no branches: run switches and the
//    forwarding of a just-updated item row (two consecutive ratings of the
//    same item, i.e. a duplicate pair) are selects, and single-lane stores
//    go through per-lane dummy addresses.
constexpr int CHUNK = 64;

struct LdsLayout {
    size_t q_off, bi_off, rec_off, p_off, bu_off, dummy_off, total;
};

__host__ __device__ inline LdsLayout lds_layout(int k, int64_t cb) {
    LdsLayout L;
    size_t o = 0;
    L.q_off = o;
    o += (size_t)cb * k * 4;
    L.bi_off = o;
    o += (size_t)cb * 4 + 64 * 4 * 4;  // slack: full-width reads of the last row stay inside
    o = (o + 15) & ~size_t(15);
    L.rec_off = o;
    o += 3 * CHUNK * sizeof(Rec);  // records: triple buffer (wave 0 reads c, helpers read c-1, write c+1)
    L.p_off = o;
    o += (size_t)2 * CHUNK * k * 4 + 64 * 4 * 4;
    L.bu_off = o;
    o += 2 * CHUNK * 4;
    L.dummy_off = o;
    o += 64 * 16 * 4;
    L.total = o;
    return L;
}

// One block of ratings [beg, end) of the processing order, whose users
// start at u0 and whose item slice starts at i0.  Called by every thread of
// a workgroup of NW waves; smem holds lds_layout(k, cb).total bytes.
template <int KPL, bool FULL, int NW>
__device__ __forceinline__ void process_block(const Rec *__restrict__ recs, int64_t beg, int64_t end, int64_t u0,
                                              int64_t i0, int64_t n, int64_t cb, int ibits, int k, float *P,
                                              float *Q, float *bu, float *bi, float mu, const HP &hp,
                                              unsigned char *smem) {
    constexpr int WG = NW * WAVE;
    constexpr int NH = NW - 1;                  // helper waves
    constexpr int PER = (CHUNK + NH - 1) / NH;  // record slots per helper wave
    const LdsLayout L = lds_layout(k, cb);
    float *Qs = reinterpret_cast<float *>(smem + L.q_off);
    float *bis = reinterpret_cast<float *>(smem + L.bi_off);
    Rec *rbuf = reinterpret_cast<Rec *>(smem + L.rec_off);
    float *Ps = reinterpret_cast<float *>(smem + L.p_off);
    float *bus = reinterpret_cast<float *>(smem + L.bu_off);
    float *dummy = reinterpret_cast<float *>(smem + L.dummy_off);

    if (beg == end) return;
    const int ncols = (int)std::min<int64_t>(cb, n - i0);
    const uint32_t imask = (1u << ibits) - 1u;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE;
    const int64_t cnt = end - beg;
    const int nchunks = (int)((cnt + CHUNK - 1) / CHUNK);

    // stage the item slice
    for (int64_t x = tid; x < (int64_t)ncols * k; x += WG) Qs[x] = Q[i0 * k + x];
    for (int x = tid; x < ncols; x += WG) bis[x] = bi[i0 + x];

    // Helper wave hw owns records l = hw + NH*jj of every chunk (the same
    // slots for write-back and staging, so its LDS reads of a slot precede
    // its writes in program order).
    const int hw = wave - 1;
    const int lj = hw + NH * lane;  // this lane's record slot

    // write back the user rows whose run ended in chunk c (buffer c & 1);
    // `next_ul` is the local user of the record after the chunk (or ~0)
    auto write_back = [&](int c, uint32_t next_ul) {
        const int buf = c & 1;
        const Rec *rb3 = rbuf + (c % 3) * CHUNK;
        const int64_t cbeg = beg + (int64_t)c * CHUNK;
        const int len = (int)std::min<int64_t>(CHUNK, end - cbeg);
        const bool valid = lane < PER && lj < len;
        uint32_t ul = 0, ul_next = next_ul;
        if (valid) {
            ul = rb3[lj].ui >> ibits;
            if (lj + 1 < len) ul_next = rb3[lj + 1].ui >> ibits;
        }
        const bool run_end = valid && ul_next != ul;
        if (run_end) bu[u0 + ul] = bus[buf * CHUNK + lj];
        const uint64_t emask = __ballot(run_end);
#pragma unroll
        for (int jj = 0; jj < PER; ++jj) {
            if ((emask >> jj) & 1ull) {
                const int l = hw + NH * jj;
                const int64_t urow = u0 + (int64_t)__builtin_amdgcn_readlane(ul, jj);
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    if (FULL || f < k) P[urow * k + f] = Ps[((size_t)buf * CHUNK + l) * k + f];
                }
            }
        }
    };

    // stage chunk c into buffer c & 1: every P row a run starts with is
    // loaded into registers before any is written, so the loads overlap
    auto stage = [&](int c) {
        const int buf = c & 1;
        const int64_t cbeg = beg + (int64_t)c * CHUNK;
        const int len = (int)std::min<int64_t>(CHUNK, end - cbeg);
        const bool valid = lane < PER && lj < len;
        uint32_t ui = 0, uprev = 0xffffffffu;
        float rr = 0.f;
        if (valid) {
            const Rec rc = recs[cbeg + lj];
            ui = rc.ui;
            rr = rc.r;
            if (lj > 0) uprev = recs[cbeg + lj - 1].ui >> ibits;
        }
        const uint32_t ul = ui >> ibits;
        const bool start = valid && (lj == 0 || uprev != ul);
        const float buv = start ? bu[u0 + ul] : 0.f;
        const uint64_t smask = __ballot(start);
        float v[PER][KPL];
#pragma unroll
        for (int jj = 0; jj < PER; ++jj) {
            if ((smask >> jj) & 1ull) {
                const int64_t urow = u0 + (int64_t)__builtin_amdgcn_readlane(ul, jj);
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    v[jj][cc] = (FULL || f < k) ? P[urow * k + f] : 0.f;
                }
            }
        }
        if (valid) {
            rbuf[(c % 3) * CHUNK + lj] = Rec{ui, rr - mu};  // the rating minus mu, as every kernel forms it first
            if (start) bus[buf * CHUNK + lj] = buv;
        }
#pragma unroll
        for (int jj = 0; jj < PER; ++jj) {
            if ((smask >> jj) & 1ull) {
                const int l = hw + NH * jj;
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    if (FULL || f < k) Ps[((size_t)buf * CHUNK + l) * k + f] = v[jj][cc];
                }
            }
        }
    };
    if (wave > 0) stage(0);
    __syncthreads();

    // wave 0 state carried across chunks
    float p[KPL], q_upd[KPL];
#pragma unroll
    for (int cc = 0; cc < KPL; ++cc) p[cc] = q_upd[cc] = 0.f;
    float bu_cur = 0.f, bi_upd = 0.f;
    uint32_t cur_ul = 0xffffffffu;

    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (wave > 0) {
            if (c > 0) {
                const uint32_t nxt = rbuf[(c % 3) * CHUNK].ui >> ibits;  // first record of chunk c
                write_back(c - 1, nxt);
            }
            if (c + 1 < nchunks) stage(c + 1);
        } else {
            const int64_t cbeg = beg + (int64_t)c * CHUNK;
            const int len = __builtin_amdgcn_readfirstlane((int)std::min<int64_t>(CHUNK, end - cbeg));
            const Rec myrec = rbuf[(c % 3) * CHUNK + lane];  // slots past len hold stale records, never used
            const uint32_t rec_ui = myrec.ui;
            const float rec_r = myrec.r;
            float *Pbuf = Ps + (size_t)buf * CHUNK * k;
            float *Bbuf = bus + buf * CHUNK;

            // rating 0 of the chunk: item row and bias (the slice already
            // holds every earlier update), staged user row
            uint32_t ui_n = __builtin_amdgcn_readlane(rec_ui, 0);
            float r_n = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rec_r), 0));
            float qn[KPL], pn[KPL];
#pragma unroll
            for (int cc = 0; cc < KPL; ++cc) {
                const int f = lane + WAVE * cc;
                const float a = Qs[(ui_n & imask) * k + f];
                const float bb = Pbuf[f];
                qn[cc] = (FULL || f < k) ? a : 0.f;
                pn[cc] = (FULL || f < k) ? bb : 0.f;
            }
            float bin = bis[ui_n & imask];
            float bun = Bbuf[0];
            bool same_item = false;
            bool new_user = (ui_n >> ibits) != cur_ul;

            for (int l = 0; l < len; ++l) {
                const uint32_t ui = ui_n;
                const uint32_t il = ui & imask;
                const float r = r_n;
                float q[KPL];
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    q[cc] = same_item ? q_upd[cc] : qn[cc];
                    p[cc] = new_user ? pn[cc] : p[cc];
                }
                const float bi0 = same_item ? bi_upd : bin;
                const float bu0 = new_user ? bun : bu_cur;
                // one rating ahead
                const int ln = (l + 1 < len) ? l + 1 : l;
                ui_n = __builtin_amdgcn_readlane(rec_ui, ln);
                r_n = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rec_r), ln));
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    const float a = Qs[(ui_n & imask) * k + f];
                    const float bb = Pbuf[(size_t)ln * k + f];
                    qn[cc] = (FULL || f < k) ? a : 0.f;
                    pn[cc] = (FULL || f < k) ? bb : 0.f;
                }
                bin = bis[ui_n & imask];
                bun = Bbuf[ln];
                same_item = (ui_n & imask) == il;
                new_user = (ui_n >> ibits) != (ui >> ibits);
                // the update (same operations as the reference kernel)
                const float cres = (r - bu0) - bi0;  // r already holds rating - mu
                const float dot = wave_sum_perm(lane_dot(p, q));
                const float e = cres - dot;
                factor_update(p, q, e, hp);
                bi_upd = bias_update(bi0, e, hp.a_bi, hp.b_bi);
                bu_cur = bias_update(bu0, e, hp.a_bu, hp.b_bu);
#pragma unroll
                for (int cc = 0; cc < KPL; ++cc) {
                    const int f = lane + WAVE * cc;
                    q_upd[cc] = q[cc];
                    float *qa = (FULL || f < k) ? &Qs[il * k + f] : &dummy[lane];
                    float *pa = (FULL || f < k) ? &Pbuf[(size_t)l * k + f] : &dummy[lane];
                    *qa = q[cc];
                    *pa = p[cc];
                }
                {
                    float *ba = lane == 0 ? &bis[il] : &dummy[lane];
                    float *ua = lane == 0 ? &Bbuf[l] : &dummy[64 + lane];
                    *ba = bi_upd;
                    *ua = bu_cur;
                }
            }
            cur_ul = __builtin_amdgcn_readlane(rec_ui, len - 1) >> ibits;
        }
        __syncthreads();
    }
    // the last chunk's runs all end here
    if (wave > 0) write_back(nchunks - 1, 0xffffffffu);
    __syncthreads();
    for (int64_t x = tid; x < (int64_t)ncols * k; x += WG) Q[i0 * k + x] = Qs[x];
    for (int x = tid; x < ncols; x += WG) bi[i0 + x] = bis[x];
}

// One stratum s: workgroup j owns block ((j + s) mod b, j).
template <int KPL, bool FULL, int NW>
__global__ __launch_bounds__(NW *WAVE) void sgd_lds_kernel(const Rec *__restrict__ recs,
                                                           const int64_t *__restrict__ block_ptr, int b, int s,
                                                           int64_t n, int64_t rb, int64_t cb, int ibits, int k,
                                                           float *P, float *Q, float *bu, float *bi, float mu,
                                                           HP hp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int j = blockIdx.x;
    const int br = (j + s) % b;
    const int64_t blk = (int64_t)br * b + j;
    process_block<KPL, FULL, NW>(recs, block_ptr[blk], block_ptr[blk + 1], (int64_t)br * rb, (int64_t)j * cb, n, cb,
                                 ibits, k, P, Q, bu, bi, mu, hp, smem);
}

// ------------------------------------------------------------- batched
// Many independent problems trained together.  Global position t of problem
// p is epoch t / b_p, position t % b_p of that epoch's stratum order; one
// launch runs position t of every problem that has one: workgroup g takes
// item items[first + g] = (problem, t, stratum s, column j) and runs block
// ((j + s) mod b_p, j) of that problem.  Blocks of one position of one
// problem form a stratum (no shared row or column); blocks of different
// problems share nothing; successive positions are ordered by the stream.
template <int KPL, bool FULL, int NW>
__global__ __launch_bounds__(NW *WAVE) void sgd_positions_kernel(const BatchProblem *__restrict__ probs,
                                                                 const BatchItem *__restrict__ items, int k,
                                                                 HP hp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchItem it = items[blockIdx.x];
    const BatchProblem pr = probs[it.p];
    const int r = (it.j + it.s) % pr.b;
    const int64_t blk = (int64_t)r * pr.b + it.j;
    process_block<KPL, FULL, NW>(pr.recs, pr.block_ptr[blk], pr.block_ptr[blk + 1], (int64_t)r * pr.rb,
                                 (int64_t)it.j * pr.cb, pr.n, pr.cb, pr.ibits, k, pr.P, pr.Q, pr.bu, pr.bi, pr.mu, hp,
                                 smem);
}

// ---------------------------------------------------------------- host
template <int KPL>
static void launch_global(Model &M, int s, const HP &hp) {
    const Partition &Pt = M.part;
    sgd_global_kernel<KPL><<<M.b, 64, 0, M.stream>>>(Pt.recs.as<Rec>(), Pt.block_ptr.as<int64_t>(), M.b, s, Pt.rb,
                                                      Pt.cb, Pt.ibits, M.k, M.P.as<float>(), M.Q.as<float>(),
                                                      M.bu.as<float>(), M.bi.as<float>(), (float)M.mu, hp);
    BMF_HIP(hipGetLastError());
}

template <class F>
static void set_max_lds(F *fn, size_t bytes) {
    BMF_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <int KPL, bool FULL, int NW>
static void launch_lds(Model &M, int s, const HP &hp, size_t lds_bytes) {
    static size_t attr_done = 0;  // per instantiation
    if (lds_bytes > attr_done) {
        set_max_lds(sgd_lds_kernel<KPL, FULL, NW>, lds_bytes);
        attr_done = lds_bytes;
    }
    const Partition &Pt = M.part;
    sgd_lds_kernel<KPL, FULL, NW><<<M.b, NW * WAVE, lds_bytes, M.stream>>>(
        Pt.recs.as<Rec>(), Pt.block_ptr.as<int64_t>(), M.b, s, M.n, Pt.rb, Pt.cb, Pt.ibits, M.k, M.P.as<float>(),
        M.Q.as<float>(), M.bu.as<float>(), M.bi.as<float>(), (float)M.mu, hp);
    BMF_HIP(hipGetLastError());
}

size_t sgd_lds_bytes(int k, int64_t cb) { return lds_layout(k, cb).total; }

int sgd_max_lds(int device) {
    static int cached[64] = {0};
    if (device < 64 && cached[device]) return cached[device];
    int v = 0;
    BMF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (device < 64) cached[device] = v;
    return v;
}

// LDS-staged kernels exist for k <= 128 (one or two factors per lane).
static bool lds_kernel_ok(int k, int nw) { return k <= 128 && (nw == 4 || nw == 8); }

static void launch_one(Model &M, int s, const HP &hp, int variant, size_t lds) {
    const int kpl = (M.k + WAVE - 1) / WAVE;
    const bool full = M.k == WAVE * kpl;
    if (variant == 2) {
        const int key = (kpl - 1) * 4 + (full ? 2 : 0) + (M.waves == 8 ? 1 : 0);
        switch (key) {
        case 0: launch_lds<1, false, 4>(M, s, hp, lds); return;
        case 1: launch_lds<1, false, 8>(M, s, hp, lds); return;
        case 2: launch_lds<1, true, 4>(M, s, hp, lds); return;
        case 3: launch_lds<1, true, 8>(M, s, hp, lds); return;
        case 4: launch_lds<2, false, 4>(M, s, hp, lds); return;
        case 5: launch_lds<2, false, 8>(M, s, hp, lds); return;
        case 6: launch_lds<2, true, 4>(M, s, hp, lds); return;
        case 7: launch_lds<2, true, 8>(M, s, hp, lds); return;
        default: break;
        }
    }
    switch (kpl) {
    case 1: launch_global<1>(M, s, hp); break;
    case 2: launch_global<2>(M, s, hp); break;
    case 3: launch_global<3>(M, s, hp); break;
    case 4: launch_global<4>(M, s, hp); break;
    case 5: launch_global<5>(M, s, hp); break;
    case 6: launch_global<6>(M, s, hp); break;
    case 7: launch_global<7>(M, s, hp); break;
    case 8: launch_global<8>(M, s, hp); break;
    default: launch_global<16>(M, s, hp); break;
    }
}

void sgd_epoch(Model &M, const int32_t *order, const HP &hp) {
    const size_t lds = sgd_lds_bytes(M.k, M.part.cb);
    const bool fits = lds_kernel_ok(M.k, M.waves) && (int64_t)lds <= sgd_max_lds(M.device);
    int variant = M.sgd_kernel;
    if (variant == 0) variant = fits ? 2 : 1;
    if (variant == 2 && !fits)
        BMF_FAIL(BMF_E_STATE, "the LDS-staged SGD kernel needs k <= 128 and an item slice that fits in LDS; use "
                              "SGD kernel 1 or a larger b");
    hipEvent_t ev0 = take_event(M), ev1 = take_event(M);
    BMF_HIP(hipEventRecord(ev0, M.stream));
    for (int pos = 0; pos < M.b; ++pos) launch_one(M, order[pos], hp, variant, lds);
    BMF_HIP(hipEventRecord(ev1, M.stream));
    M.pending.emplace_back(ev0, ev1);
    M.sgd_launches += M.b;
    if (M.pending.size() > 64) harvest_timing(M, false);
}

template <int KPL, bool FULL, int NW>
static void launch_positions(const BatchProblem *d_probs, const BatchItem *d_items, int64_t count, int k,
                             const HP &hp, size_t lds, hipStream_t s) {
    static size_t attr_done = 0;
    if (lds > attr_done) {
        set_max_lds(sgd_positions_kernel<KPL, FULL, NW>, lds);
        attr_done = lds;
    }
    sgd_positions_kernel<KPL, FULL, NW><<<(unsigned)count, NW * WAVE, lds, s>>>(d_probs, d_items, k, hp);
    BMF_HIP(hipGetLastError());
}

void sgd_positions_launch(int k, int nw, const BatchProblem *d_probs, const BatchItem *d_items, int64_t count,
                          const HP &hp, size_t lds, hipStream_t s) {
    if (count == 0) return;
    if (!lds_kernel_ok(k, nw)) BMF_FAIL(BMF_E_INVAL, "batched training needs k <= 128 and 4 or 8 waves per block");
    const int kpl = (k + WAVE - 1) / WAVE;
    const bool full = k == WAVE * kpl;
    const int key = (kpl - 1) * 4 + (full ? 2 : 0) + (nw == 8 ? 1 : 0);
    switch (key) {
    case 0: launch_positions<1, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 1: launch_positions<1, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 2: launch_positions<1, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 3: launch_positions<1, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 4: launch_positions<2, false, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    case 5: launch_positions<2, false, 8>(d_probs, d_items, count, k, hp, lds, s); break;
    case 6: launch_positions<2, true, 4>(d_probs, d_items, count, k, hp, lds, s); break;
    default: launch_positions<2, true, 8>(d_probs, d_items, count, k, hp, lds, s); break;
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
