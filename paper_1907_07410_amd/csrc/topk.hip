// Top-K recommendation scoring: for each requested user, the K items with
// the largest predicted rating mu + bu_u + bi_i + p_u . q_i (Eq 3 plus the
// global mean), ties to the smaller item id.
//
// The score matrix users x items is the one dense contraction of the
// method, so it runs on MFMA and is never stored: each wave multiplies 16
// users against 16-item tiles and filters every score against the user's
// running K-th best, appending survivors to an LDS candidate buffer that is
// compacted (sorted, cut to K) when it fills.
//
//   FP32 path: v_mfma_f32_16x16x4_f32 on the FP32 factors.
//   BF16 path: v_mfma_f32_16x16x32_bf16 on round-to-nearest-even BF16
//              copies (FP32 accumulate) picks Kc candidates, which are then
//              rescored with FP32 factors and cut to K.
//
// The latent index order inside an MFMA tile is fixed and independent of
// the users sharing the tile, so a user's scores (and hence its result) do
// not depend on the rest of the batch.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "wave.h"

namespace bmf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TU = 16;  // users per wave (MFMA N)
constexpr int TI = 16;  // items per tile (MFMA M)

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// ------------------------------------------------------------ bf16 tables
__global__ void bf16_table_kernel(const float *__restrict__ A, int64_t rows, int k, int kb, uint16_t *__restrict__ out) {
    const int64_t total = rows * kb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / kb;
        const int f = (int)(t % kb);
        out[t] = f < k ? to_bf16_rne(A[row * k + f]) : (uint16_t)0;
    }
}

// Gather the requested users' rows: FP32 (stride kp, zero padded), BF16
// (stride kb) and the per-user offset mu + bu_u.  Invalid ids get a zero
// vector and a NaN offset (their rows decode to item -1).
__global__ void gather_users_kernel(const int32_t *__restrict__ users, int64_t nu, int64_t nu_pad, int64_t m,
                                    const float *__restrict__ P, const float *__restrict__ bu, float mu, int k,
                                    int kp, int kb, float *__restrict__ Ug, uint16_t *__restrict__ Ugb,
                                    float *__restrict__ ub) {
    const int64_t total = nu_pad * kb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / kb;
        const int f = (int)(t % kb);
        const int64_t u = q < nu ? (int64_t)users[q] : -1;
        const bool ok = u >= 0 && u < m;
        const float v = (ok && f < k) ? P[u * k + f] : 0.f;
        if (f < kp) Ug[q * kp + f] = v;
        if (Ugb) Ugb[q * kb + f] = to_bf16_rne(v);
        if (f == 0) ub[q] = ok ? mu + bu[u] : __int_as_float(0x7fc00000);
    }
}

// ------------------------------------------------------ score + select
template <int CAP>
struct SelShared {
    uint64_t cand[TU][CAP];
    int cnt[TU];
};

// Sort the first `size` keys of buf descending (bitonic network, all
// comparators descending; positions at or past size act as key 0, the
// worst key, and are never touched).  One wave; LDS accesses of a wave are
// performed in order, so no barrier is needed between steps.
__device__ __forceinline__ void wave_sort_desc(uint64_t *buf, int size) {
    int N = 1;
    while (N < size) N <<= 1;
    const int lane = __lane_id();
    for (int p = 2; p <= N; p <<= 1) {
        const int half = p >> 1;
        for (int idx = lane; idx < N / 2; idx += WAVE) {
            const int x = (idx / half) * p + (idx % half);
            const int y = (idx / half) * p + p - 1 - (idx % half);
            if (y < size) {
                const uint64_t a = buf[x], c = buf[y];
                if (a < c) {
                    buf[x] = c;
                    buf[y] = a;
                }
            }
        }
        for (int q = half >> 1; q >= 1; q >>= 1) {
            for (int idx = lane; idx < N / 2; idx += WAVE) {
                const int x = (idx / q) * 2 * q + (idx % q);
                const int y = x + q;
                if (y < size) {
                    const uint64_t a = buf[x], c = buf[y];
                    if (a < c) {
                        buf[x] = c;
                        buf[y] = a;
                    }
                }
            }
        }
    }
}

template <int KC, int CAP, bool BF16>
__global__ __launch_bounds__(64) void score_select_kernel(const float *__restrict__ Ug, const uint16_t *__restrict__ Ugb,
                                                          const float *__restrict__ Qf,
                                                          const uint16_t *__restrict__ Qb,
                                                          const float *__restrict__ bi, int64_t n, int k, int kp,
                                                          int kb, int K, int64_t per_split, int S,
                                                          uint64_t *__restrict__ out) {
    __shared__ SelShared<CAP> sh;
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int split = blockIdx.y;
    const int64_t ibeg = (int64_t)split * per_split;
    const int64_t iend = std::min<int64_t>(n, ibeg + per_split);
    const int ucol = lane % 16, grp = lane / 16;
    const int64_t urow = tile * TU + ucol;

    if (lane < TU) sh.cnt[lane] = 0;
    float thr = -INFINITY;  // threshold of user ucol

    // user operand fragments in registers
    f32x4 bf[BF16 ? 1 : KC];
    bf16x8 bb[BF16 ? KC : 1];
    if (!BF16) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            bf[c] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (c * 16 < kp) bf[c] = *reinterpret_cast<const f32x4 *>(Ug + urow * kp + c * 16 + 4 * grp);
        }
    } else {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            uint4 raw = {0u, 0u, 0u, 0u};
            if (c * 32 < kb) raw = *reinterpret_cast<const uint4 *>(Ugb + urow * kb + c * 32 + 8 * grp);
            bb[c] = __builtin_bit_cast(bf16x8, raw);
        }
    }

    for (int64_t ib = ibeg; ib < iend; ib += TI) {
        const int64_t irow = ib + ucol;  // item row this lane feeds into the A operand
        const bool irow_ok = irow < iend;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        if (!BF16) {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                f32x4 a = {0.f, 0.f, 0.f, 0.f};
                const int f0 = c * 16 + 4 * grp;
                if (irow_ok) {
                    if (f0 + 3 < k && (k & 3) == 0) {
                        a = *reinterpret_cast<const f32x4 *>(Qf + irow * k + f0);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) a[e] = (f0 + e < k) ? Qf[irow * k + f0 + e] : 0.f;
                    }
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], bf[c][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], bf[c][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], bf[c][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], bf[c][3], acc, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                uint4 raw = {0u, 0u, 0u, 0u};
                if (irow_ok && c * 32 < kb) raw = *reinterpret_cast<const uint4 *>(Qb + irow * kb + c * 32 + 8 * grp);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, raw), bb[c], acc, 0, 0, 0);
            }
        }
        // lane holds items ib + 4*grp + r for user ucol
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t item = ib + 4 * grp + r;
            if (item < iend) {
                const float s = acc[r] + bi[item];
                if (s > thr) {
                    const int pos = atomicAdd(&sh.cnt[ucol], 1);
                    sh.cand[ucol][pos] = rank_key(s, (int32_t)item);
                }
            }
        }
        // compact users whose buffer could overflow on the next tile
        const int my = lane < TU ? sh.cnt[lane] : 0;
        uint64_t full = __ballot(lane < TU && my > CAP - 16);
        while (full) {
            const int uu = __builtin_ctzll(full);
            full &= full - 1;
            const int c = sh.cnt[uu];
            wave_sort_desc(sh.cand[uu], c);
            if (lane == 0) sh.cnt[uu] = std::min(c, K);
            // new threshold: K-th best key's score
            const float t = key_score(sh.cand[uu][K - 1]);
            if (ucol == uu) thr = t;
        }
    }
    // final: sort every user's buffer and emit K keys (0 = empty)
    for (int uu = 0; uu < TU; ++uu) {
        const int c = sh.cnt[uu];
        wave_sort_desc(sh.cand[uu], c);
        const int64_t row = tile * TU + uu;
        uint64_t *o = out + (row * S + split) * (int64_t)K;
        for (int j = lane; j < K; j += WAVE) o[j] = j < c ? sh.cand[uu][j] : 0ull;
    }
}

// Merge the S partial lists of each user (S*K keys, each list already
// sorted) into the best Kout keys.  One workgroup per user.
constexpr int MERGE_WG = 256;
constexpr int MERGE_CAP = 8192;

__global__ __launch_bounds__(MERGE_WG) void merge_kernel(const uint64_t *__restrict__ part, int S, int K, int Kout,
                                                         uint64_t *__restrict__ out) {
    __shared__ uint64_t buf[MERGE_CAP];
    const int64_t row = blockIdx.x;
    const int total = S * K;
    for (int x = threadIdx.x; x < total; x += MERGE_WG) buf[x] = part[row * total + x];
    __syncthreads();
    int N = 1;
    while (N < total) N <<= 1;
    for (int p = 2; p <= N; p <<= 1) {
        const int half = p >> 1;
        for (int idx = threadIdx.x; idx < N / 2; idx += MERGE_WG) {
            const int x = (idx / half) * p + (idx % half);
            const int y = (idx / half) * p + p - 1 - (idx % half);
            if (y < total) {
                const uint64_t a = buf[x], c = buf[y];
                if (a < c) {
                    buf[x] = c;
                    buf[y] = a;
                }
            }
        }
        __syncthreads();
        for (int q = half >> 1; q >= 1; q >>= 1) {
            for (int idx = threadIdx.x; idx < N / 2; idx += MERGE_WG) {
                const int x = (idx / q) * 2 * q + (idx % q);
                const int y = x + q;
                if (y < total) {
                    const uint64_t a = buf[x], c = buf[y];
                    if (a < c) {
                        buf[x] = c;
                        buf[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < Kout; j += MERGE_WG) out[row * Kout + j] = j < total ? buf[j] : 0ull;
}

// FP32 rescore of Kc candidates per user, then the best K.  One wave per
// user; lane f owns factors f, f+64, ...; each candidate's dot product is a
// fixed-order butterfly (same every call).
template <int KPL>
__global__ __launch_bounds__(64) void rescore_kernel(const uint64_t *__restrict__ cand, int Kc, int K,
                                                     const float *__restrict__ Ug, int kp,
                                                     const float *__restrict__ Qf, const float *__restrict__ bi,
                                                     int k, uint64_t *__restrict__ out) {
    __shared__ uint64_t buf[2048];
    const int64_t row = blockIdx.x;
    const int lane = threadIdx.x;
    float p[KPL];
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
        const int f = lane + WAVE * c;
        p[c] = f < k ? Ug[row * kp + f] : 0.f;
    }
    for (int j = 0; j < Kc; ++j) {
        const uint64_t key = cand[row * Kc + j];
        uint64_t nk = 0ull;
        if (key != 0ull) {
            const int32_t item = key_item(key);
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < KPL; ++c) {
                const int f = lane + WAVE * c;
                const float qv = f < k ? Qf[(int64_t)item * k + f] : 0.f;
                d = c == 0 ? p[c] * qv : fmaf(p[c], qv, d);
            }
            d = wave_sum_xor(d);
            nk = rank_key(d + bi[item], item);
        }
        if (lane == 0) buf[j] = nk;
    }
    wave_sort_desc(buf, Kc);
    for (int j = lane; j < K; j += WAVE) out[row * K + j] = j < Kc ? buf[j] : 0ull;
}

__global__ void decode_kernel(const uint64_t *__restrict__ keys, int64_t nu, int K, const float *__restrict__ ub,
                              int32_t *__restrict__ items, float *__restrict__ scores) {
    const int64_t total = nu * K;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / K;
        const uint64_t key = keys[t];
        const float off = ub[q];
        if (key == 0ull || off != off) {
            items[t] = -1;
            scores[t] = -INFINITY;
        } else {
            items[t] = key_item(key);
            scores[t] = off + key_score(key);
        }
    }
}

// ------------------------------------------------------------------ host
static int cap_for(int K) {
    if (K + 16 <= 192) return 256;
    if (K + 16 <= 448) return 512;
    return 1024;
}

template <int KC, bool BF16>
static void launch_select(int cap, dim3 grid, const float *Ug, const uint16_t *Ugb, const float *Qf, const uint16_t *Qb,
                          const float *bi, int64_t n, int k, int kp, int kb, int K, int64_t per_split, int S,
                          uint64_t *out, hipStream_t s) {
    switch (cap) {
    case 256:
        score_select_kernel<KC, 256, BF16><<<grid, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out);
        break;
    case 512:
        score_select_kernel<KC, 512, BF16><<<grid, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out);
        break;
    default:
        score_select_kernel<KC, 1024, BF16><<<grid, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out);
        break;
    }
    BMF_HIP(hipGetLastError());
}

template <bool BF16>
static void select_dispatch(int kc, int cap, dim3 grid, const float *Ug, const uint16_t *Ugb, const float *Qf,
                            const uint16_t *Qb, const float *bi, int64_t n, int k, int kp, int kb, int K,
                            int64_t per_split, int S, uint64_t *out, hipStream_t s) {
    switch (kc) {
    case 1: launch_select<1, BF16>(cap, grid, Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out, s); break;
    case 2: launch_select<2, BF16>(cap, grid, Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out, s); break;
    case 3:
    case 4: launch_select<4, BF16>(cap, grid, Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out, s); break;
    case 5: case 6: case 7:
    case 8: launch_select<8, BF16>(cap, grid, Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out, s); break;
    default: launch_select<16, BF16>(cap, grid, Ug, Ugb, Qf, Qb, bi, n, k, kp, kb, K, per_split, S, out, s); break;
    }
}

void ensure_bf16_items(Model &M) {
    if (M.bf16_valid) return;
    const int kb = round_up(M.k, 32);
    const size_t need = (size_t)M.n * kb * sizeof(uint16_t);
    if (M.Qb.bytes < need) M.Qb.alloc(need);
    const int grid = (int)std::min<int64_t>((M.n * kb + 255) / 256, 8192);
    bf16_table_kernel<<<grid, 256, 0, M.stream>>>(M.Q.as<float>(), M.n, M.k, kb, M.Qb.as<uint16_t>());
    BMF_HIP(hipGetLastError());
    M.bf16_valid = true;
}

TopkPlan topk_plan(const Model &M, int64_t nu, int K, int precision, int Kc) {
    TopkPlan T;
    T.nu = nu;
    T.K = K;
    T.bf = precision == 1;
    T.Ksel = T.bf ? topk_candidates(K, Kc) : K;
    T.kp = round_up(M.k, 16);
    T.kb = round_up(M.k, 32);
    T.nu_pad = (nu + TU - 1) / TU * TU;
    const int64_t tiles = T.nu_pad / TU;
    // item splits: enough workgroups to fill the chip, merged afterwards
    int S = (int)std::max<int64_t>(1, (2048 + tiles - 1) / std::max<int64_t>(tiles, 1));
    S = (int)std::min<int64_t>(S, std::max<int64_t>(1, M.n / 256));
    S = std::min(S, std::max(1, MERGE_CAP / T.Ksel));
    T.per_split = ((M.n + S - 1) / S + TI - 1) / TI * TI;
    T.S = (int)std::max<int64_t>(1, (M.n + T.per_split - 1) / T.per_split);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += (bytes + 255) & ~size_t(255);
        return at;
    };
    T.off_ug = take((size_t)T.nu_pad * T.kp * 4);
    T.off_ugb = take((size_t)T.nu_pad * T.kb * 2);
    T.off_ub = take((size_t)T.nu_pad * 4);
    T.off_part = take((size_t)T.nu_pad * T.S * T.Ksel * 8);
    T.off_sel = take((size_t)T.nu_pad * std::max(T.Ksel, T.K) * 8);
    T.total = o;
    return T;
}

void topk_gather(Model &M, const TopkPlan &T, const int32_t *d_users, unsigned char *work, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((T.nu_pad * T.kb + 255) / 256, 8192);
    gather_users_kernel<<<grid, 256, 0, s>>>(d_users, T.nu, T.nu_pad, M.m, M.P.as<float>(), M.bu.as<float>(),
                                            (float)M.mu, M.k, T.kp, T.kb, reinterpret_cast<float *>(work + T.off_ug),
                                            T.bf ? reinterpret_cast<uint16_t *>(work + T.off_ugb) : nullptr,
                                            reinterpret_cast<float *>(work + T.off_ub));
    BMF_HIP(hipGetLastError());
}

void topk_score(Model &M, const TopkPlan &T, unsigned char *work, int32_t *d_items, float *d_scores, hipStream_t s) {
    if (T.nu == 0) return;
    const float *Ug = reinterpret_cast<const float *>(work + T.off_ug);
    const uint16_t *Ugb = reinterpret_cast<const uint16_t *>(work + T.off_ugb);
    const float *ub = reinterpret_cast<const float *>(work + T.off_ub);
    uint64_t *part = reinterpret_cast<uint64_t *>(work + T.off_part);
    uint64_t *sel = reinterpret_cast<uint64_t *>(work + T.off_sel);
    const int cap = cap_for(T.Ksel);
    const dim3 grid((unsigned)(T.nu_pad / TU), (unsigned)T.S);
    if (T.bf) {
        if (!M.bf16_valid) BMF_FAIL(BMF_E_STATE, "BF16 item table not prepared");
        select_dispatch<true>(T.kb / 32, cap, grid, Ug, Ugb, M.Q.as<float>(), M.Qb.as<uint16_t>(), M.bi.as<float>(),
                              M.n, M.k, T.kp, T.kb, T.Ksel, T.per_split, T.S, part, s);
    } else {
        select_dispatch<false>(T.kp / 16, cap, grid, Ug, Ugb, M.Q.as<float>(), nullptr, M.bi.as<float>(), M.n, M.k,
                               T.kp, T.kb, T.Ksel, T.per_split, T.S, part, s);
    }
    const uint64_t *cand = part;
    if (T.S > 1) {
        merge_kernel<<<(unsigned)T.nu, MERGE_WG, 0, s>>>(part, T.S, T.Ksel, T.Ksel, sel);
        BMF_HIP(hipGetLastError());
        cand = sel;
    }
    const uint64_t *fin = cand;
    if (T.bf) {
        uint64_t *dst = (cand == sel) ? part : sel;
        const int kpl = (M.k + 63) / 64;
#define RS_LAUNCH(KPL)                                                                                              \
    rescore_kernel<KPL><<<(unsigned)T.nu, 64, 0, s>>>(cand, T.Ksel, T.K, Ug, T.kp, M.Q.as<float>(), M.bi.as<float>(), \
                                                      M.k, dst)
        switch (kpl) {
        case 1: RS_LAUNCH(1); break;
        case 2: RS_LAUNCH(2); break;
        case 3: RS_LAUNCH(3); break;
        default: RS_LAUNCH(4); break;
        }
#undef RS_LAUNCH
        BMF_HIP(hipGetLastError());
        fin = dst;
    }
    const int dgrid = (int)std::min<int64_t>((T.nu * T.K + 255) / 256, 8192);
    decode_kernel<<<dgrid, 256, 0, s>>>(fin, T.nu, T.K, ub, d_items, d_scores);
    BMF_HIP(hipGetLastError());
}

void topk_run(Model &M, const int32_t *d_users, int64_t nu, int K, int precision, int Kc, int32_t *d_items,
              float *d_scores) {
    if (nu == 0) return;
    if (M.k > 256) BMF_FAIL(BMF_E_INVAL, "top-K scoring supports k <= 256");
    const TopkPlan T = topk_plan(M, nu, K, precision, Kc);
    if (M.scratch.bytes < T.total) M.scratch.alloc(T.total);
    unsigned char *w = M.scratch.as<unsigned char>();
    topk_gather(M, T, d_users, w, M.stream);
    if (T.bf) ensure_bf16_items(M);
    topk_score(M, T, w, d_items, d_scores, M.stream);
}

}  // namespace bmf
