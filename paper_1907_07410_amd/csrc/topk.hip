// Top-K recommendation scoring: for each requested user, the K items with
// the largest predicted rating mu + bu_u + bi_i + p_u . q_i (Eq 3 plus the
// global mean), ties to the smaller item id.
//
// The score matrix users x items is the one dense contraction of the
// method, so it runs on MFMA and is never stored; the work that remains is
// selection.  Three passes per request:
//  1. threshold: the r-th best of each user's scores against a fixed sample
//     of s = 1024 evenly spaced item ids (rounded down in its last 8 key
//     bits), r chosen so that the chance that fewer than the needed number
//     of items reach it is below 1e-6 (no threshold when n <= 1024: every
//     item is a candidate);
//  2. filter: the full user x item contraction, split over the item range
//     across workgroups; every score at or above the user's threshold goes
//     through a per-lane list in LDS to the user's candidate buffer in
//     global memory, sized so that it overflows for about 1 user in 1e9;
//  3. finish: one wave per user keeps the candidates that can be among the
//     best (a histogram cut), sorts them and keeps the best.
// A user whose buffer got fewer than the needed candidates (or overflowed,
// or whose scores tie too often to be cut) is redone by the full-selection
// kernel (scores filtered against a running K-th best in an LDS buffer over
// all items), launched every time and exiting at once when no user of its
// tile needs it.  The result is exact in every case: the best items of the
// candidates are the best items overall whenever enough items reach the
// threshold.
//
//   FP32 path: v_mfma_f32_16x16x4_f32 on the FP32 factors.
//   BF16 path: v_mfma_f32_16x16x32_bf16 on round-to-nearest-even BF16
//              copies (FP32 accumulate) picks Kc candidates, which are then
//              rescored with FP32 factors and cut to K; the finish and the
//              rescore are one kernel, which rescores only the candidates
//              that a bound on the BF16 rounding leaves able to reach the
//              FP32 top K (the answer equals rescoring all Kc).
//   BF16 only: the BF16 path's ranking with its BF16 scores, K candidates
//              and no rescore.
//
// The latent index order inside an MFMA tile is fixed and independent of
// the users sharing the tile, and a user's threshold and candidates depend
// on its own scores only, so a user's result does not depend on the rest of
// the batch.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>

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
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------ bf16 tables
__global__ void bf16_table_kernel(const float *__restrict__ A, int64_t rows, int k, int kb, uint16_t *__restrict__ out) {
    const int64_t total = rows * kb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / kb;
        const int f = (int)(t % kb);
        out[t] = f < k ? to_bf16_rne(A[row * k + f]) : (uint16_t)0;
    }
}

// Per-item bounds used by the BF16 path's candidate drop: qn[2 j] >=
// ||Q_j||_2 and qn[2 j + 1] >= ||bf16(Q_j) - Q_j||_2 (the difference is
// exact in FP32; both norms inflated by 1e-4 relative, more than their
// rounding for k <= 256).  One wave per row.
__global__ void item_norms_kernel(const float *__restrict__ Q, int64_t n, int k, float *__restrict__ qn) {
    const int lane = threadIdx.x % WAVE;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t j = w0; j < n; j += nw) {
        float s2 = 0.f, d2 = 0.f;
        for (int f = lane; f < k; f += WAVE) {
            const float v = Q[j * k + f];
            const float d = bf16_value(to_bf16_rne(v)) - v;
            s2 = fmaf(v, v, s2);
            d2 = fmaf(d, d, d2);
        }
        s2 = wave_sum_xor(s2);
        d2 = wave_sum_xor(d2);
        if (lane == 0) {
            qn[2 * j] = sqrtf(s2) * 1.0001f;
            qn[2 * j + 1] = sqrtf(d2) * 1.0001f;
        }
    }
}

// Gather the requested users' rows: FP32 (stride kp, zero padded), BF16
// (stride kb) and the per-user offset mu + bu_u.  Invalid ids get a zero
// vector and a NaN offset (their rows decode to item -1).
__global__ void gather_users_kernel(const int32_t *__restrict__ users, int64_t nu, int64_t nu_pad, int64_t m,
                                    const float *__restrict__ P, const float *__restrict__ bu, float mu, int k,
                                    int kp, int kb, float *__restrict__ Ug, uint16_t *__restrict__ Ugb,
                                    float *__restrict__ ub) {
    // one wave per row, four factors per lane per turn (kp and kb are
    // multiples of 16 and 32, so a lane's four stay inside both rows)
    const int lane = threadIdx.x % WAVE;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t q = w0; q < nu_pad; q += nw) {
        const int64_t u = q < nu ? (int64_t)users[q] : -1;
        const bool ok = u >= 0 && u < m;
        for (int f = 4 * lane; f < kb; f += 4 * WAVE) {
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (ok && (k & 3) == 0 && f < k) {
                const float4 x = *reinterpret_cast<const float4 *>(P + u * k + f);
                v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
            } else if (ok) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = f + e < k ? P[u * k + f + e] : 0.f;
            }
            if (f < kp) *reinterpret_cast<float4 *>(Ug + q * kp + f) = float4{v[0], v[1], v[2], v[3]};
            if (Ugb) {
                const uint32_t lo = (uint32_t)to_bf16_rne(v[0]) | (uint32_t)to_bf16_rne(v[1]) << 16;
                const uint32_t hi = (uint32_t)to_bf16_rne(v[2]) | (uint32_t)to_bf16_rne(v[3]) << 16;
                *reinterpret_cast<uint2 *>(Ugb + q * kb + f) = uint2{lo, hi};
            }
        }
        if (lane == 0) ub[q] = ok ? mu + bu[u] : __int_as_float(0x7fc00000);
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
    int lgN = 0;
    while ((1 << lgN) < size) ++lgN;
    const int half_n = (1 << lgN) >> 1;
    const int lane = __lane_id();
    for (int lp = 1; lp <= lgN; ++lp) {
        const int lh = lp - 1;  // log2 of half the merged run
        for (int idx = lane; idx < half_n; idx += WAVE) {
            const int lo = idx & ((1 << lh) - 1);
            const int x = ((idx >> lh) << lp) + lo;
            const int y = ((idx >> lh) << lp) + (1 << lp) - 1 - lo;
            if (y < size) {
                const uint64_t a = buf[x], c = buf[y];
                if (a < c) {
                    buf[x] = c;
                    buf[y] = a;
                }
            }
        }
        for (int lq = lh - 1; lq >= 0; --lq) {
            for (int idx = lane; idx < half_n; idx += WAVE) {
                const int x = ((idx >> lq) << (lq + 1)) + (idx & ((1 << lq) - 1));
                const int y = x + (1 << lq);
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

// User operand fragments of a 16-user tile (rows of Ug / Ugb).
template <int KC, bool BF16>
struct UserFrag {
    f32x4 f[BF16 ? 1 : KC];
    bf16x8 b[BF16 ? KC : 1];
    // chunks c0 .. c0 + KC - 1 of the row (16 factors each in FP32, 32 in BF16)
    __device__ __forceinline__ void load(const float *Ug, const uint16_t *Ugb, int64_t urow, int kp, int kb, int grp,
                                         int c0 = 0) {
        if (!BF16) {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                f[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                if ((c0 + c) * 16 < kp) f[c] = *reinterpret_cast<const f32x4 *>(Ug + urow * kp + (c0 + c) * 16 + 4 * grp);
            }
        } else {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                uint4 raw = {0u, 0u, 0u, 0u};
                if ((c0 + c) * 32 < kb) raw = *reinterpret_cast<const uint4 *>(Ugb + urow * kb + (c0 + c) * 32 + 8 * grp);
                b[c] = __builtin_bit_cast(bf16x8, raw);
            }
        }
    }
};

// A operand of a 16-item tile: this lane's part of item row `irow` (zero
// when !irow_ok).  Split from the MFMAs so that loops can load the next
// tile while the current one is multiplied.
template <int KC, bool BF16>
struct ItemFrag {
    f32x4 f[BF16 ? 1 : KC];
    uint4 b[BF16 ? KC : 1];
    __device__ __forceinline__ void load(const float *__restrict__ Qf, const uint16_t *__restrict__ Qb, int64_t irow,
                                         bool irow_ok, int k, int kb, int grp, int c0 = 0) {
        if (!BF16) {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                f32x4 a = {0.f, 0.f, 0.f, 0.f};
                const int f0 = (c0 + c) * 16 + 4 * grp;
                if (irow_ok) {
                    if (f0 + 3 < k && (k & 3) == 0) {
                        a = *reinterpret_cast<const f32x4 *>(Qf + irow * k + f0);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) a[e] = (f0 + e < k) ? Qf[irow * k + f0 + e] : 0.f;
                    }
                }
                f[c] = a;
            }
        } else {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                uint4 raw = {0u, 0u, 0u, 0u};
                if (irow_ok && (c0 + c) * 32 < kb)
                    raw = *reinterpret_cast<const uint4 *>(Qb + irow * kb + (c0 + c) * 32 + 8 * grp);
                b[c] = raw;
            }
        }
    }
};

// Dot products of a 16-item x 16-user tile: acc[r] = score of user
// (lane % 16) with item (tile item 4 * (lane / 16) + r), accumulated onto
// the given start (the item biases where the caller wants whole scores).
template <int KC, bool BF16>
__device__ __forceinline__ f32x4 tile_mma(const UserFrag<KC, BF16> &U, const ItemFrag<KC, BF16> &A,
                                          f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f}) {
    if (!BF16) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][0], U.f[c][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][1], U.f[c][1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][2], U.f[c][2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][3], U.f[c][3], acc, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int c = 0; c < KC; ++c)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A.b[c]), U.b[c], acc, 0, 0, 0);
    }
    return acc;
}

// Chunk c of tile_mma alone (16 factors in FP32: four MFMAs; 32 in BF16:
// one): tile_mma is these for c = 0 .. KC - 1 in turn.
template <int KC, bool BF16>
__device__ __forceinline__ f32x4 tile_mma_chunk(const UserFrag<KC, BF16> &U, const ItemFrag<KC, BF16> &A, int c,
                                                f32x4 acc) {
    if (!BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][0], U.f[c][0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][1], U.f[c][1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][2], U.f[c][2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.f[c][3], U.f[c][3], acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A.b[c]), U.b[c], acc, 0, 0, 0);
    }
    return acc;
}

template <int KC, bool BF16>
__device__ __forceinline__ f32x4 tile_dots(const UserFrag<KC, BF16> &U, const float *__restrict__ Qf,
                                           const uint16_t *__restrict__ Qb, int64_t irow, bool irow_ok, int k,
                                           int kb, int grp, f32x4 start) {
    ItemFrag<KC, BF16> A;
    A.load(Qf, Qb, irow, irow_ok, k, kb, grp);
    return tile_mma(U, A, start);
}

constexpr int SAMPLE_MAX = 1024;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, WAVE));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, WAVE));
    return v;
}

// Pass 1: threshold per user: the r-th best of its scores over the sample
// items t * n / s, t < s, rounded down (so at least r sampled items reach
// it).  One sweep stores the sampled scores of the tile's 16 users in LDS as
// ordered keys; then wave w finds user w's r-th largest key bit by bit, from
// the top: a bit is kept when at least r keys reach the value with it set.
// The bits above the highest one in which the smallest and the largest key
// differ are those two keys' common bits, and the search stops above the
// lowest SMP_LOW_BITS bits (left zero: the threshold is at most 2^-15 of its
// value below the exact r-th key, so it admits a few more items).  The filter
// scores a sampled item exactly as this pass does (the same MFMA tile and
// bias), so the r sampled items at or above the threshold pass it there too.
// Stored as an ordered key; 0 = no threshold (r = 0).  Also clears the
// user's candidate count.  One workgroup of SMP_WAVES waves per 16-user tile,
// each wave taking every SMP_WAVES-th sample tile in the sweep; lane (u, g)
// holds user u's scores.  The pass fits 64 registers (no row prefetch;
// fragments in pieces of up to 4 chunks), so two workgroups share a CU and
// one's selection overlaps the other's sweep.
constexpr int SMP_WAVES = 16;
constexpr int SMP_LOW_BITS = 8;
static_assert(SMP_WAVES == TU, "one wave per user of the tile selects its threshold");

template <int KC, bool BF16>
__global__ __launch_bounds__(SMP_WAVES *WAVE, 8) void sample_threshold_kernel(
    const float *__restrict__ Ug, const uint16_t *__restrict__ Ugb, const float *__restrict__ Qf,
    const uint16_t *__restrict__ Qb, const float *__restrict__ bi, int64_t n, int k, int kp, int kb, int s, int r,
    uint32_t *__restrict__ thr, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t keys[TU][SAMPLE_MAX];
    const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
    const int64_t tile = blockIdx.x;
    const int ucol = lane % 16, grp = lane / 16;
    if (tid < TU) cnt[tile * TU + tid] = 0u;
    if (r == 0) {
        if (tid < TU) thr[tile * TU + tid] = 0u;
        return;
    }
    const int step = SMP_WAVES * TI;
    auto sample_bias = [&](int t0, float (&b)[4]) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int t = t0 + 4 * grp + rr;
            b[rr] = t < s ? bi[(int64_t)t * n / s] : 0.f;
        }
    };
    // the wave's sample tiles; user and item fragments in pieces of H <= 4
    // chunks (the user's loaded once when there is one piece), multiplied in
    // the same order as one tile_mma over all KC chunks
    constexpr int H = KC > 4 ? 4 : KC;
    UserFrag<H, BF16> U;
    if (H == KC) U.load(Ug, Ugb, tile * TU + ucol, kp, kb, grp);
    for (int t0 = wave * TI; t0 < s; t0 += step) {
        const int ta = t0 + ucol;
        float b[4];
        sample_bias(t0, b);
        f32x4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
        for (int h = 0; h < KC / H; ++h) {
            if (H != KC) U.load(Ug, Ugb, tile * TU + ucol, kp, kb, grp, h * H);
            ItemFrag<H, BF16> A;
            A.load(Qf, Qb, (int64_t)ta * n / s, ta < s, k, kb, grp, h * H);
            acc = tile_mma(U, A, acc);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int t = t0 + 4 * grp + rr;
            if (t < s) keys[ucol][t] = float_to_ordered(acc[rr]);
        }
    }
    __syncthreads();
    // wave w: user w's r-th largest key
    const uint32_t *mine = keys[wave];
    constexpr int PER = SAMPLE_MAX / WAVE;
    uint32_t kv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int t = lane + WAVE * j;
        kv[j] = t < s ? mine[t] : 0u;  // 0: below every real key, never counted
    }
    uint32_t lo = ~0u, hi = 0u;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (lane + WAVE * j < s) lo = min(lo, kv[j]);
        hi = max(hi, kv[j]);
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    // every key lies in [lo, hi], so the r-th largest shares their common
    // high bits; the search sets the rest from the highest differing bit
    const uint32_t diff = lo ^ hi;
    const int top = diff ? 31 - __builtin_clz(diff) : SMP_LOW_BITS - 1;
    uint32_t ans = top >= 31 ? 0u : hi & ~((2u << top) - 1u);
    for (int bit = top; bit >= SMP_LOW_BITS; --bit) {
        const uint32_t cand = ans | (1u << bit);
        int c = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) c += __popcll(__ballot(kv[j] >= cand));
        if (c >= r) ans = cand;
    }
    if (!diff) ans = hi & ~((1u << SMP_LOW_BITS) - 1u);
    if (lane == 0) thr[tile * TU + wave] = ans;
}

// Pass 2: every score at or above its user's threshold goes to the user's
// candidate buffer (capg keys; the count keeps growing past capg so that an
// overflow is seen).  Grid: groups of UT user tiles x item splits (the split
// varying fastest); a wave holds the user fragments of its UT tiles, so each
// item tile it loads feeds UT tile products (UT times fewer item-table reads
// than one tile per wave).  Tiles at or beyond `tiles` are skipped.
// Candidates gather in LDS in per-lane lists: a lane holds four scores of
// one user per tile product (items 4 grp .. 4 grp + 3 of the tile, user
// ucol), and appends each one that reaches the user's threshold to its own
// list for that user tile, FLT_SUB entries of {score, item offset in the
// split}, with the list length in a register.  Every score is written at
// the list's end and only a passing one moves the end, so the append takes
// no branch and no atomic.  Entry e of lane l in list q sits at
// (q FLT_SUB + e) WAVE + l: a wave's writes at any mix of list lengths
// fall in distinct banks.  A tile adds at most 4 to a list, so when some
// list of a user tile holds more than FLT_SUB - 4 after a tile, the four
// lists of each of that tile's users go to the global buffer (one counter
// reservation per user); the rest goes there at the end.
// User tiles per filter wave.
static constexpr int filter_tiles_per_wave(int kc, bool bf16) {
    return bf16 ? (kc == 4 ? 4 : kc <= 8 ? 2 : 1) : (kc == 8 ? 4 : kc <= 4 ? 2 : 1);
}
// List entries per lane and user tile: two filter workgroups per SIMD (8
// per CU) leave each 20 KB of the CU's 160 KB of LDS; the lists take 18 KB.
template <int UT>
constexpr int filter_sub() {
    return 18 * 1024 / (UT * WAVE * 8);
}

// Raw buffer resource over `bytes` bytes from `base`: a load at an offset
// at or past `bytes` returns zeros and touches no memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// FAST: the item rows are whole 16-byte chunks (BF16 rows padded to kb, or
// FP32 rows with k = 16 KC), read through a buffer resource clipped to the
// split's rows, so a tile's loads need no per-lane address arithmetic and
// no bounds branch; otherwise plain loads with bounds tests.
template <int KC, bool BF16, int UT, bool FAST>
__global__ __launch_bounds__(64, 2) void filter_kernel(const float *__restrict__ Ug, const uint16_t *__restrict__ Ugb,
                                                    const float *__restrict__ Qf, const uint16_t *__restrict__ Qb,
                                                    const float *__restrict__ bi, int64_t n, int k, int kp, int kb,
                                                    int64_t tiles, int64_t per_split, int splits,
                                                    const uint32_t *__restrict__ thr, uint32_t *__restrict__ cnt,
                                                    int capg, uint64_t *__restrict__ cand) {
    constexpr int SUB = filter_sub<UT>();
    static_assert(SUB >= 8, "lists too short for the LDS budget");
    // scores in the first half, item offsets in the second
    constexpr int HALF = UT * SUB * WAVE;
    __shared__ uint32_t lst[2 * HALF];
    const int lane = threadIdx.x;
    // the item split varies fastest with the workgroup id: workgroups are
    // dealt to the XCDs in turn, so with a multiple of 8 splits each XCD's L2
    // holds the item rows of its own splits only
    const int64_t tile0 = (int64_t)(blockIdx.x / splits) * UT;
    const int64_t ibeg = (int64_t)(blockIdx.x % splits) * per_split;
    const int64_t iend = std::min<int64_t>(n, ibeg + per_split);
    const int ucol = lane % 16, grp = lane / 16;
    const int nt = (int)std::min<int64_t>(UT, tiles - tile0);  // wave-uniform
    UserFrag<KC, BF16> U[UT];
    // thresholds as floats: sv >= tf passes every score whose ordered key
    // reaches the threshold (and, at most, a -0 against a +0 threshold too);
    // no threshold (0) passes every number, and a NaN (an item beyond the
    // range) nothing.  A user tile beyond the last gets a NaN threshold: its
    // scores (those of tile 0 again) pass nothing, so its lists stay empty
    // and the loop needs no test for it.
    float tf[UT];
    // the end of this lane's list of each user tile, as an index into lst
    int end[UT];
#pragma unroll
    for (int q = 0; q < UT; ++q) {
        const int64_t urow = (tile0 + (q < nt ? q : 0)) * TU + ucol;
        U[q].load(Ug, Ugb, urow, kp, kb, grp);
        const uint32_t t = thr[urow];
        tf[q] = q >= nt ? __builtin_nanf("") : t == 0u ? -INFINITY : ordered_to_float(t);
        end[q] = q * SUB * WAVE + lane;
    }
    // user tile q's lists to the global buffer: the four lanes of a user
    // (ucol + 16 g) add up their lengths, the first reserves the total with
    // one returning atomic, and each copies its list behind the lists of
    // the lanes before it.  One wave per workgroup: its LDS accesses happen
    // in program order.
    auto flush = [&](int q) {
        const int first = q * SUB * WAVE + lane;
        const int c = (end[q] - first) / WAVE;
        const int c_pair = __shfl_xor(c, 16);
        const int s2 = c + c_pair;
        const int s2_other = __shfl_xor(s2, 32);
        const int total = s2 + s2_other;
        const int before = ((grp & 1) ? c_pair : 0) + ((grp & 2) ? s2_other : 0);
        const int64_t urow = (tile0 + q) * TU + ucol;
        uint32_t g = 0u;
        if (grp == 0 && total > 0) g = atomicAdd(&cnt[urow], (uint32_t)total);
        g = __shfl(g, ucol);
        for (int e = 0; e < c; ++e) {
            const uint32_t at = g + (uint32_t)(before + e);
            if (at < (uint32_t)capg)
                cand[urow * capg + at] =
                    rank_key(__uint_as_float(lst[first + e * WAVE]), (int32_t)(ibeg + lst[HALF + first + e * WAVE]));
        }
        end[q] = first;
    };
    // one tile's scores, with the item bias as the accumulator's start; the
    // UT products chunk by chunk, so that consecutive MFMAs are independent
    // (each product's own chunk order is that of tile_mma)
    auto products = [&](const ItemFrag<KC, BF16> &A, const f32x4 &b, f32x4 (&acc)[UT]) {
#pragma unroll
        for (int q = 0; q < UT; ++q) acc[q] = b;
#pragma unroll
        for (int c = 0; c < KC; ++c)
#pragma unroll
            for (int q = 0; q < UT; ++q) acc[q] = tile_mma_chunk(U[q], A, c, acc[q]);
    };
    // every score of tile ib is written at its list's end and only a passing
    // one moves the end; then the lists that a further tile could overflow
    // are flushed
    auto append = [&](int64_t ib, f32x4 (&acc)[UT], bool whole) {
        if (!whole && ib + TI > iend) {
            // rows past the split read as zeros: no score there
            const int64_t left = iend - ib;
#pragma unroll
            for (int q = 0; q < UT; ++q)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    if (4 * grp + rr >= left) acc[q][rr] = __builtin_nanf("");
        }
        const uint32_t off = (uint32_t)(ib - ibeg) + 4u * (uint32_t)grp;
        // the UT lists advance side by side (independent chains)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int q = 0; q < UT; ++q) {
                const int e = end[q];
                lst[e] = __float_as_uint(acc[q][rr]);
                lst[HALF + e] = off + (uint32_t)rr;
                end[q] = e + (acc[q][rr] >= tf[q] ? WAVE : 0);
            }
        bool full = false;
#pragma unroll
        for (int q = 0; q < UT; ++q) full |= end[q] > (q * SUB + SUB - 4) * WAVE + lane;
        if (__ballot(full)) {
#pragma unroll
            for (int q = 0; q < UT; ++q)
                if (__ballot(end[q] > (q * SUB + SUB - 4) * WAVE + lane)) flush(q);
        }
    };
    if constexpr (FAST) {
        // this lane's 16 bytes of chunk c of its tile row (row ucol, bytes
        // 16 grp of the chunk's 64): the same offsets in FP32 and in BF16
        const unsigned char *qb = BF16 ? reinterpret_cast<const unsigned char *>(Qb)
                                       : reinterpret_cast<const unsigned char *>(Qf);
        const uint32_t rowb = BF16 ? (uint32_t)kb * 2u : (uint32_t)k * 4u;
        const uint32_t lq = (uint32_t)ucol * rowb + 16u * (uint32_t)grp;
        auto load = [&](int64_t ib, ItemFrag<KC, BF16> &A, f32x4 &b) {
            const int64_t at = std::min<int64_t>(ib, iend);
            const uint32_t rows = (uint32_t)std::min<int64_t>(iend - at, TI);
            const __amdgpu_buffer_rsrc_t rq = raw_rsrc(qb + at * rowb, rows * rowb);
            const __amdgpu_buffer_rsrc_t rb = raw_rsrc(bi + at, rows * 4u);
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const auto raw = __builtin_amdgcn_raw_buffer_load_b128(rq, lq + 64u * (uint32_t)c, 0, 0);
                if (BF16)
                    A.b[c] = __builtin_bit_cast(uint4, raw);
                else
                    A.f[c] = __builtin_bit_cast(f32x4, raw);
            }
            b = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, 16u * (uint32_t)grp, 0, 0));
        };
        // each tile's rows are loaded one tile ahead of its products; two
        // buffers alternate
        ItemFrag<KC, BF16> A0, A1;
        f32x4 b0, b1;
        f32x4 acc[UT];
        load(ibeg, A0, b0);
        for (int64_t ib = ibeg;;) {
            load(ib + TI, A1, b1);
            products(A0, b0, acc);
            append(ib, acc, ib + TI <= iend);
            ib += TI;
            if (ib >= iend) break;
            load(ib + TI, A0, b0);
            products(A1, b1, acc);
            append(ib, acc, ib + TI <= iend);
            ib += TI;
            if (ib >= iend) break;
        }
    } else {
        // item biases of this lane's four score items of a tile (items
        // 4 grp .. 4 grp + 3, 16-byte aligned): one load on a whole tile, NaN
        // beyond the range
        auto load_bias = [&](int64_t ib, f32x4 &b) {
            const int64_t item = ib + 4 * grp;
            if (ib + TI <= iend) {
                b = *reinterpret_cast<const f32x4 *>(bi + item);
            } else {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) b[rr] = item + rr < iend ? bi[item + rr] : __builtin_nanf("");
            }
        };
        ItemFrag<KC, BF16> A, An;
        f32x4 b, bn;
        A.load(Qf, Qb, ibeg + ucol, ibeg + ucol < iend, k, kb, grp);
        load_bias(ibeg, b);
        bn = b;
        for (int64_t ib = ibeg; ib < iend; ib += TI) {
            // the next tile's rows and biases, loaded while this one is multiplied
            const int64_t inext = ib + TI + ucol;
            An.load(Qf, Qb, inext, inext < iend, k, kb, grp);
            if (ib + TI < iend) load_bias(ib + TI, bn);
            f32x4 acc[UT];
            products(A, b, acc);
            append(ib, acc, false);
            A = An;
            b = bn;
        }
    }
#pragma unroll
    for (int q = 0; q < UT; ++q)
        if (q < nt) flush(q);
}

// The latent chunk count the pass kernels are instantiated for.
static int dispatch_kc(int kc) { return kc <= 2 ? kc : kc <= 4 ? 4 : kc <= 8 ? 8 : 16; }

// Pass 3: one wave per user keeps the candidates that can be among its best
// `need` (a 256-bin histogram of their scores between the smallest and the
// largest gives a cut bin; every key in the cut bin and above is kept),
// sorts those (descending keys) and writes the best `need` (0 = none).  A
// user with fewer than `need` candidates under a real threshold, with an
// overflowed buffer, or with more than KEEP - need keys whose score ties the
// need-th best (a cut bin holding too many keys is first narrowed by an
// exact selection of that score) is marked in fail[] for the full-selection
// kernel.  The wave
// reads its candidates from the global buffer once per phase (the reads
// after the first hit in the caches) and needs no workgroup barrier.
constexpr int FIN_WG = WAVE;
constexpr int CAPG_MAX = 8192;
constexpr int FIN_BINS = 256;
constexpr int FIN_KEEP = 1024;  // >= the largest `need` (1008)
// LDS for the kept keys: 512 when need <= FIN_KEEP_SMALL_NEED (room for the
// cut bin's extra keys), else FIN_KEEP
constexpr int FIN_KEEP_SMALL = 512, FIN_KEEP_SMALL_NEED = 384;
static_assert(FIN_BINS == 4 * WAVE, "four bins per lane");

// Orders this wave's LDS accesses before and after the call (LDS operations
// of one wave are performed in issue order; this keeps the compiler from
// moving them across).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The histogram cut of one user's candidates by one wave: every key that
// can be among the best `need` goes to buf (the first KEEP of them; the
// return value is the kept count, which exceeds KEEP only when more than
// KEEP - need keys tie with the need-th best).  edge_rank gets a
// lower bound on the high half of the key of rank `rank` (<= need): the
// smallest high half of the bins that hold the best `rank` keys (0 when
// total <= need and no histogram was made).
template <int KEEP>
__device__ __forceinline__ int fin_cut(const uint64_t *__restrict__ mine, int total, int need, int rank,
                                       uint64_t *buf, uint32_t *hist, uint32_t &edge_rank) {
    const int lane = threadIdx.x;
    edge_rank = 0u;
    if (total <= need) {
        for (int x = lane; x < total; x += WAVE) buf[x] = mine[x];
        return total;
    }
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int x = lane; x < total; x += WAVE) {
        const uint32_t h = (uint32_t)(mine[x] >> 32);
        lo = min(lo, h);
        hi = max(hi, h);
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    // histogram of the score halves over [lo, hi] in 256 equal bins; the cut
    // bin is the highest one with at least `need` keys in it and above, so
    // every key of the best `need` is in a kept bin
    const uint64_t span = (uint64_t)(hi - lo) + 1u;
    auto bin_of = [&](uint64_t key) { return (int)(((uint64_t)((uint32_t)(key >> 32) - lo) * FIN_BINS) / span); };
#pragma unroll
    for (int e = 0; e < 4; ++e) hist[4 * lane + e] = 0u;
    wave_lds_fence();
    for (int x = lane; x < total; x += WAVE) atomicAdd(&hist[bin_of(mine[x])], 1u);
    wave_lds_fence();
    uint32_t h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = hist[4 * lane + e];
    // suffix sums from the top bin down: lanes above this one first
    const uint32_t own = h[0] + h[1] + h[2] + h[3];
    uint32_t above = own;  // inclusive suffix over lanes >= this one
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_down((int)above, d, WAVE);
        if (lane + d < WAVE) above += o;
    }
    uint32_t suf = above - own;  // keys in the bins above this lane's four
    // this lane's bins whose suffix reaches need, resp. rank (the suffix only
    // falls with the bin, so bins 0 .. cut are the ones that do)
    uint32_t nb = 0u;
#pragma unroll
    for (int e = 3; e >= 0; --e) {
        suf += h[e];
        nb += (suf >= (uint32_t)need ? 1u : 0u) + (suf >= (uint32_t)rank ? 1u << 16 : 0u);
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) nb += (uint32_t)__shfl_xor((int)nb, off, WAVE);
    const int cut = (int)(nb & 0xFFFFu) - 1, cut_rank = (int)(nb >> 16) - 1;
    // a key is in bin cut_rank or above when its high half reaches
    // lo + ceil(cut_rank * span / 256)
    edge_rank = lo + (uint32_t)(((uint64_t)cut_rank * span + FIN_BINS - 1) / FIN_BINS);
    // compaction: every key of the cut bin and above, in candidate order
    int m = 0;
    for (int x0 = 0; x0 < total; x0 += WAVE) {
        const int x = x0 + lane;
        uint64_t key = 0ull;
        bool keep = false;
        if (x < total) {
            key = mine[x];
            keep = bin_of(key) >= cut;
        }
        const uint64_t bal = __ballot(keep);
        const int at = m + __popcll(bal & ((1ull << lane) - 1ull));
        if (keep && at < KEEP) buf[at] = key;
        m += __popcll(bal);
    }
    if (m <= KEEP) return m;
    // The cut bin holds too many keys (a few far scores stretch the bins):
    // the high half of the need-th best key, bit by bit from the top (a bit
    // stays when at least need keys reach the value with it set), and every
    // key at or above it -- need plus the keys tied with it.  No rank edge on
    // this path.
    uint32_t hq = 0u;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t c1 = hq | (1u << bit);
        uint32_t c = 0u;
        for (int x = lane; x < total; x += WAVE) c += (uint32_t)(mine[x] >> 32) >= c1 ? 1u : 0u;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) c += (uint32_t)__shfl_xor((int)c, off, WAVE);
        if (c >= (uint32_t)need) hq = c1;
    }
    edge_rank = 0u;
    m = 0;
    for (int x0 = 0; x0 < total; x0 += WAVE) {
        const int x = x0 + lane;
        uint64_t key = 0ull;
        bool keep = false;
        if (x < total) {
            key = mine[x];
            keep = (uint32_t)(key >> 32) >= hq;
        }
        const uint64_t bal = __ballot(keep);
        const int at = m + __popcll(bal & ((1ull << lane) - 1ull));
        if (keep && at < KEEP) buf[at] = key;
        m += __popcll(bal);
    }
    return m;
}

template <int KEEP>
__global__ __launch_bounds__(FIN_WG) void finish_kernel(const uint32_t *__restrict__ thr,
                                                        const uint32_t *__restrict__ cnt,
                                                        const uint64_t *__restrict__ cand, int capg, int need,
                                                        uint32_t *__restrict__ fail, uint64_t *__restrict__ sel) {
    __shared__ uint64_t buf[KEEP];
    __shared__ uint32_t hist[FIN_BINS];
    const int lane = threadIdx.x;
    const int64_t row = blockIdx.x;
    const uint32_t c = cnt[row];
    const bool ok = c <= (uint32_t)capg && (c >= (uint32_t)need || thr[row] == 0u);
    if (!ok) {
        if (lane == 0) fail[row] = 1u;
        return;
    }
    uint32_t edge;
    const int m = fin_cut<KEEP>(cand + row * (int64_t)capg, (int)c, need, need, buf, hist, edge);
    if (m > KEEP) {
        if (lane == 0) fail[row] = 1u;
        return;
    }
    if (lane == 0) fail[row] = 0u;
    wave_lds_fence();
    wave_sort_desc(buf, m);
    wave_lds_fence();
    for (int j = lane; j < need; j += WAVE) sel[row * need + j] = j < m ? buf[j] : 0ull;
}

// Full selection for the users marked in fail[] (all items): each score is
// compared with the user's running K-th best and survivors go to an LDS
// buffer that is sorted and cut to K when it fills.  One wave per 16-user
// tile; a tile with no marked user returns at once.
template <int KC, int CAP, bool BF16>
__global__ __launch_bounds__(64) void score_select_kernel(const float *__restrict__ Ug, const uint16_t *__restrict__ Ugb,
                                                          const float *__restrict__ Qf,
                                                          const uint16_t *__restrict__ Qb,
                                                          const float *__restrict__ bi, int64_t n, int k, int kp,
                                                          int kb, int K, const uint32_t *__restrict__ fail,
                                                          uint64_t *__restrict__ out) {
    __shared__ SelShared<CAP> sh;
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int ucol = lane % 16, grp = lane / 16;
    const int64_t urow = tile * TU + ucol;
    if (__ballot(lane < TU && fail[tile * TU + lane] != 0u) == 0ull) return;

    if (lane < TU) sh.cnt[lane] = 0;
    float thr = -INFINITY;  // threshold of user ucol
    UserFrag<KC, BF16> U;
    U.load(Ug, Ugb, urow, kp, kb, grp);

    for (int64_t ib = 0; ib < n; ib += TI) {
        const int64_t irow = ib + ucol;
        f32x4 bias;
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[r] = ib + 4 * grp + r < n ? bi[ib + 4 * grp + r] : 0.f;
        // the scores as the filter forms them (the bias as the start)
        const f32x4 acc = tile_dots<KC, BF16>(U, Qf, Qb, irow, irow < n, k, kb, grp, bias);
        // lane holds items ib + 4*grp + r for user ucol
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t item = ib + 4 * grp + r;
            if (item < n) {
                const float s = acc[r];
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
    // final: sort every marked user's buffer and emit K keys (0 = empty)
    for (int uu = 0; uu < TU; ++uu) {
        const int64_t row = tile * TU + uu;
        if (fail[row] == 0u) continue;
        const int c = sh.cnt[uu];
        wave_sort_desc(sh.cand[uu], c);
        uint64_t *o = out + row * (int64_t)K;
        for (int j = lane; j < K; j += WAVE) o[j] = j < c ? sh.cand[uu][j] : 0ull;
    }
}

// FP32 rescoring of BF16 candidates.  One wave per user; its four 16-lane
// groups take one candidate each at a time, and lane l of a group multiplies
// the factor chunks 4 (l + 16 c) .. + 3 (c = 0, 1, ...) in one fma chain,
// then the group sums its lanes with the fixed butterfly of row16_sum.  A
// candidate's item row is read by one group in one pass (16 lanes x 16
// contiguous bytes per load), and the summation order is the same every
// call and in both kernels below.
// RS_MAXC chunks of four factors per lane cover k <= 64 RS_MAXC; RS_U
// candidates per group are in flight.  Two forms: k <= 128 (2 chunks, 8
// candidates in flight) and k <= 256 (4 chunks, 4 in flight).
template <int RS_MAXC>
struct RescoreUser {
    float4 pv[RS_MAXC];     // k % 4 == 0: this lane's chunks
    float ps[4 * RS_MAXC];  // otherwise: factors l + 16 c
    __device__ __forceinline__ void load(const float *__restrict__ Ug, int64_t row, int kp, int k, int l) {
        if ((k & 3) == 0) {
#pragma unroll
            for (int c = 0; c < RS_MAXC; ++c) {
                const int f = 4 * (l + 16 * c);
                pv[c] = f < k ? *reinterpret_cast<const float4 *>(Ug + row * kp + f) : float4{0.f, 0.f, 0.f, 0.f};
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4 * RS_MAXC; ++c) {
                const int f = l + 16 * c;
                ps[c] = f < k ? Ug[row * kp + f] : 0.f;
            }
        }
    }
    // upper bounds on ||p||_2 and ||bf16(p) - p||_2 (every lane of a group
    // gets the same values; the differences are exact, the norms inflated by
    // 1e-4 relative)
    __device__ __forceinline__ void norms(int k, float &pn, float &dp) const {
        float v = 0.f, w = 0.f;
        auto add = [&](float x) {
            const float d = bf16_value(to_bf16_rne(x)) - x;
            v = fmaf(x, x, v);
            w = fmaf(d, d, w);
        };
        if ((k & 3) == 0) {
#pragma unroll
            for (int c = 0; c < RS_MAXC; ++c) {
                add(pv[c].x);
                add(pv[c].y);
                add(pv[c].z);
                add(pv[c].w);
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4 * RS_MAXC; ++c) add(ps[c]);
        }
        pn = sqrtf(row16_sum(v)) * 1.0001f;
        dp = sqrtf(row16_sum(w)) * 1.0001f;
    }
};

// Rescored keys of candidates src[j] (j = 4 t + group < R) into dst[j]
// (src and dst may be the same LDS array: a group reads its key before it
// writes the new one at the same position).  Empty keys (0) stay 0.
template <int RS_MAXC>
__device__ __forceinline__ void rescore_keys(const RescoreUser<RS_MAXC> &P, const uint64_t *src, uint64_t *dst, int R,
                                             const float *__restrict__ Qf, const float *__restrict__ bi, int k) {
    constexpr int RS_U = RS_MAXC <= 2 ? 8 : 4;
    const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
    if ((k & 3) == 0) {
        for (int j0 = 0; j0 < R; j0 += 4 * RS_U) {
            uint64_t key[RS_U];
#pragma unroll
            for (int u = 0; u < RS_U; ++u) {
                const int j = j0 + 4 * u + g;
                key[u] = j < R ? src[j] : 0ull;
            }
            float4 q[RS_U][RS_MAXC];
#pragma unroll
            for (int u = 0; u < RS_U; ++u) {
                const float *qr = Qf + (int64_t)(key[u] != 0ull ? key_item(key[u]) : 0) * k;
#pragma unroll
                for (int c = 0; c < RS_MAXC; ++c) {
                    const int f = 4 * (l + 16 * c);
                    q[u][c] = (key[u] != 0ull && f < k) ? *reinterpret_cast<const float4 *>(qr + f)
                                                        : float4{0.f, 0.f, 0.f, 0.f};
                }
            }
#pragma unroll
            for (int u = 0; u < RS_U; ++u) {
                float d = 0.f;
#pragma unroll
                for (int c = 0; c < RS_MAXC; ++c) {
                    d = fmaf(P.pv[c].x, q[u][c].x, d);
                    d = fmaf(P.pv[c].y, q[u][c].y, d);
                    d = fmaf(P.pv[c].z, q[u][c].z, d);
                    d = fmaf(P.pv[c].w, q[u][c].w, d);
                }
                d = row16_sum(d);
                const int j = j0 + 4 * u + g;
                if (l == 0 && j < R) {
                    const int32_t item = key_item(key[u]);
                    dst[j] = key[u] != 0ull ? rank_key(d + bi[item], item) : 0ull;
                }
            }
        }
    } else {
        for (int j0 = 0; j0 < R; j0 += 4) {
            const int j = j0 + g;
            const uint64_t key = j < R ? src[j] : 0ull;
            const float *qr = Qf + (int64_t)(key != 0ull ? key_item(key) : 0) * k;
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 4 * RS_MAXC; ++c) {
                const int f = l + 16 * c;
                if (key != 0ull && f < k) d = fmaf(P.ps[c], qr[f], d);
            }
            d = row16_sum(d);
            if (l == 0 && j < R) {
                const int32_t item = key_item(key);
                dst[j] = key != 0ull ? rank_key(d + bi[item], item) : 0ull;
            }
        }
    }
}

// Rescore of the users marked in fail[] (their Kc BF16 keys at sel + row *
// Kc, from the full selection), then their best K in place at sel + row *
// Kc.  Users not marked were finished by finish_rescore_kernel.
template <int RS_MAXC>
__global__ __launch_bounds__(64) void rescore_kernel(uint64_t *__restrict__ sel, int Kc, int K,
                                                     const uint32_t *__restrict__ fail,
                                                     const float *__restrict__ Ug, int kp,
                                                     const float *__restrict__ Qf, const float *__restrict__ bi,
                                                     int k) {
    __shared__ uint64_t buf[FIN_KEEP];  // Kc <= 1008
    const int64_t row = blockIdx.x;
    const int lane = threadIdx.x;
    if (fail[row] == 0u) return;
    RescoreUser<RS_MAXC> P;
    P.load(Ug, row, kp, k, lane & 15);
    uint64_t *keys = sel + row * (int64_t)Kc;
    rescore_keys(P, keys, buf, Kc, Qf, bi, k);
    wave_lds_fence();
    wave_sort_desc(buf, Kc);
    wave_lds_fence();
    for (int j = lane; j < K; j += WAVE) keys[j] = j < Kc ? buf[j] : 0ull;
}

// BF16 path, passes 3 and 4 in one: the histogram cut keeps the candidates
// that can be among the best Kc BF16 keys, and of those only the ones that
// can still reach the FP32 top K are rescored.  With B a BF16 score (the
// filter's) and F the FP32 score of the same item, |B - F| <= eps, where eps
// bounds the rounding of both operands to BF16 (relative 2^-9 each) and the
// FP32 accumulation in both kernels.  With dp = bf16(p) - p and dq =
// bf16(q) - q (exact in FP32), the exact BF16 product sum differs from the
// exact one by p.dq + dp.q + dp.dq, at most ||p|| ||dq|| + ||dp|| ||q|| +
// ||dp|| ||dq||; each FP32 sum of k + 1 terms (the MFMA's, whatever its
// order, even truncating, and the rescore's) errs by at most 2 (k + 1) 2^-24
// times the sum of the magnitudes, bounded through the same norms and |b|:
//   eps = ||p|| ||dq|| + ||dp|| ||q|| + ||dp|| ||dq||
//         + 4 (k + 2) 2^-24 ((||p|| + ||dp||)(||q|| + ||dq||) + ||p|| ||q|| + 2 |b|),
// inflated by 1%, the item terms maximised over the kept keys (which hold
// the best Kc).
// If T is the K-th best BF16 score among the candidates, K of them have
// F >= T - eps, so a kept candidate with B < T - 2 eps has F < T - eps and
// is not in the FP32 top K of the best Kc; it is dropped.
// T is bounded below by the lower edge of the histogram bin holding the
// K-th best key.  The kept keys above that bound form a prefix of the key
// order; when there are at most Kc of them they are all among the best Kc
// and only they are rescored, otherwise the best Kc are found by a sort and
// rescored.  The result equals rescoring all Kc.  A user that the cut
// cannot handle is marked in fail[] for the full selection and
// rescore_kernel.  The best K keys go to sel + row * Kc.
template <int KEEP, int RS_MAXC>
__global__ __launch_bounds__(FIN_WG) void finish_rescore_kernel(
    const uint32_t *__restrict__ thr, const uint32_t *__restrict__ cnt, const uint64_t *__restrict__ cand, int capg,
    int Kc, int K, const float *__restrict__ Ug, int kp, const float *__restrict__ Qf, const float *__restrict__ bi,
    int k, const float *__restrict__ qn, int prune, uint32_t *__restrict__ fail, uint64_t *__restrict__ sel) {
    __shared__ uint64_t buf[KEEP];
    __shared__ uint32_t hist[FIN_BINS];
    const int lane = threadIdx.x;
    const int64_t row = blockIdx.x;
    const uint32_t c = cnt[row];
    const bool ok = c <= (uint32_t)capg && (c >= (uint32_t)Kc || thr[row] == 0u);
    if (!ok) {
        if (lane == 0) fail[row] = 1u;
        return;
    }
    uint32_t edge;
    const int m = fin_cut<KEEP>(cand + row * (int64_t)capg, (int)c, Kc, K, buf, hist, edge);
    if (m > KEEP) {
        if (lane == 0) fail[row] = 1u;
        return;
    }
    if (lane == 0) fail[row] = 0u;
    RescoreUser<RS_MAXC> P;
    P.load(Ug, row, kp, k, lane & 15);
    // the drop bound (no drop without a histogram edge or when turned off)
    float lim = -INFINITY;
    if (prune && edge != 0u) {
        // the largest item norm, BF16 residual norm and |bias| among the
        // kept keys
        float qm = 0.f, dm = 0.f, bm = 0.f;
        for (int x = lane; x < m; x += WAVE) {
            const int32_t item = key_item(buf[x]);
            qm = fmaxf(qm, qn[2 * (int64_t)item]);
            dm = fmaxf(dm, qn[2 * (int64_t)item + 1]);
            bm = fmaxf(bm, fabsf(bi[item]));
        }
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            qm = fmaxf(qm, __shfl_xor(qm, off, WAVE));
            dm = fmaxf(dm, __shfl_xor(dm, off, WAVE));
            bm = fmaxf(bm, __shfl_xor(bm, off, WAVE));
        }
        float pn, dp;
        P.norms(k, pn, dp);
        const float g = 4.f * (float)(k + 2) * 0x1p-24f;
        const float eps =
            1.01f * (pn * dm + dp * qm + dp * dm + g * ((pn + dp) * (qm + dm) + pn * qm + 2.f * bm)) + 1e-30f;
        const float t = ordered_to_float(edge);
        lim = t - 2.f * eps - fabsf(t) * 0x1p-20f;
        if (!(lim == lim)) lim = -INFINITY;
    }
    wave_lds_fence();
    // keep the keys at or above lim at the front of buf, in place (a chunk's
    // keys move to positions below the next chunk's)
    int u = 0;
    for (int x0 = 0; x0 < m; x0 += WAVE) {
        const int x = x0 + lane;
        const uint64_t key = x < m ? buf[x] : 0ull;
        const bool keep = x < m && !(key_score(key) < lim);
        const uint64_t bal = __ballot(keep);
        const int at = u + __popcll(bal & ((1ull << lane) - 1ull));
        wave_lds_fence();
        if (keep) buf[at] = key;
        u += __popcll(bal);
    }
    wave_lds_fence();
    int R = u;
    if (u > Kc) {
        wave_sort_desc(buf, u);
        wave_lds_fence();
        R = Kc;
    }
    rescore_keys(P, buf, buf, R, Qf, bi, k);
    wave_lds_fence();
    wave_sort_desc(buf, R);
    wave_lds_fence();
    uint64_t *o = sel + row * (int64_t)Kc;
    for (int j = lane; j < K; j += WAVE) o[j] = j < R ? buf[j] : 0ull;
}

// The best K keys of user q at keys + q * stride to items and scores (the
// user's offset mu + bu added back; -1 / -inf for empty keys).
__global__ void decode_kernel(const uint64_t *__restrict__ keys, int64_t nu, int K, int stride,
                              const float *__restrict__ ub, int32_t *__restrict__ items, float *__restrict__ scores) {
    const int64_t total = nu * K;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / K;
        const uint64_t key = keys[q * stride + (t - q * K)];
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

// Pass kernels of one request for the given latent chunk count KC.
template <int KC, bool BF16>
static void launch_passes(const TopkPlan &T, const float *Ug, const uint16_t *Ugb, const float *Qf,
                          const uint16_t *Qb, const float *bi, int64_t n, int k, const float *qn, uint32_t *thr,
                          uint32_t *cnt, uint32_t *fail, uint64_t *cand, uint64_t *sel, hipStream_t s) {
    const unsigned tiles = (unsigned)(T.nu_pad / TU);
    sample_threshold_kernel<KC, BF16><<<tiles, SMP_WAVES * WAVE, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, T.s, T.r, thr, cnt);
    BMF_HIP(hipGetLastError());
    constexpr int UT = filter_tiles_per_wave(KC, BF16);
    if (T.ut != UT) BMF_FAIL(BMF_E_STATE, "top-K plan made for another filter shape");
    const unsigned groups = (unsigned)((tiles + UT - 1) / UT);
    if (BF16 || k == 16 * KC)
        filter_kernel<KC, BF16, UT, true><<<groups * (unsigned)T.S, 64, 0, s>>>(
            Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, (int64_t)tiles, T.per_split, T.S, thr, cnt, T.capg, cand);
    else
        filter_kernel<KC, BF16, UT, false><<<groups * (unsigned)T.S, 64, 0, s>>>(
            Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, (int64_t)tiles, T.per_split, T.S, thr, cnt, T.capg, cand);
    BMF_HIP(hipGetLastError());
    const unsigned rows = (unsigned)T.nu_pad;
    const bool small = T.Ksel <= FIN_KEEP_SMALL_NEED;
    if (BF16 && T.rescore) {
        const bool k128 = k <= 128;
        if (small && k128)
            finish_rescore_kernel<FIN_KEEP_SMALL, 2><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, T.K, Ug,
                                                                            T.kp, Qf, bi, k, qn, T.prune, fail, sel);
        else if (small)
            finish_rescore_kernel<FIN_KEEP_SMALL, 4><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, T.K, Ug,
                                                                            T.kp, Qf, bi, k, qn, T.prune, fail, sel);
        else if (k128)
            finish_rescore_kernel<FIN_KEEP, 2><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, T.K, Ug, T.kp,
                                                                      Qf, bi, k, qn, T.prune, fail, sel);
        else
            finish_rescore_kernel<FIN_KEEP, 4><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, T.K, Ug, T.kp,
                                                                      Qf, bi, k, qn, T.prune, fail, sel);
    } else {
        if (small)
            finish_kernel<FIN_KEEP_SMALL><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, fail, sel);
        else
            finish_kernel<FIN_KEEP><<<rows, FIN_WG, 0, s>>>(thr, cnt, cand, T.capg, T.Ksel, fail, sel);
    }
    BMF_HIP(hipGetLastError());
    switch (cap_for(T.Ksel)) {
    case 256:
        score_select_kernel<KC, 256, BF16><<<tiles, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, T.Ksel, fail, sel);
        break;
    case 512:
        score_select_kernel<KC, 512, BF16><<<tiles, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, T.Ksel, fail, sel);
        break;
    default:
        score_select_kernel<KC, 1024, BF16><<<tiles, 64, 0, s>>>(Ug, Ugb, Qf, Qb, bi, n, k, T.kp, T.kb, T.Ksel, fail,
                                                                 sel);
        break;
    }
    BMF_HIP(hipGetLastError());
    if (BF16 && T.rescore) {
        // the users the full selection redid
        if (k <= 128)
            rescore_kernel<2><<<(unsigned)T.nu, 64, 0, s>>>(sel, T.Ksel, T.K, fail, Ug, T.kp, Qf, bi, k);
        else
            rescore_kernel<4><<<(unsigned)T.nu, 64, 0, s>>>(sel, T.Ksel, T.K, fail, Ug, T.kp, Qf, bi, k);
        BMF_HIP(hipGetLastError());
    }
}

template <bool BF16>
static void passes_dispatch(int kc, const TopkPlan &T, const float *Ug, const uint16_t *Ugb, const float *Qf,
                            const uint16_t *Qb, const float *bi, int64_t n, int k, const float *qn, uint32_t *thr,
                            uint32_t *cnt, uint32_t *fail, uint64_t *cand, uint64_t *sel, hipStream_t s) {
    switch (kc) {
    case 1: launch_passes<1, BF16>(T, Ug, Ugb, Qf, Qb, bi, n, k, qn, thr, cnt, fail, cand, sel, s); break;
    case 2: launch_passes<2, BF16>(T, Ug, Ugb, Qf, Qb, bi, n, k, qn, thr, cnt, fail, cand, sel, s); break;
    case 3:
    case 4: launch_passes<4, BF16>(T, Ug, Ugb, Qf, Qb, bi, n, k, qn, thr, cnt, fail, cand, sel, s); break;
    case 5: case 6: case 7:
    case 8: launch_passes<8, BF16>(T, Ug, Ugb, Qf, Qb, bi, n, k, qn, thr, cnt, fail, cand, sel, s); break;
    default: launch_passes<16, BF16>(T, Ug, Ugb, Qf, Qb, bi, n, k, qn, thr, cnt, fail, cand, sel, s); break;
    }
}

// Smallest r with P(Poisson(lambda) >= r) <= eps: a sample of s items out of
// n holds about lambda = need * s / n of the best `need` items, so the r-th
// best sampled score is at most the need-th best overall except with
// probability eps.
static int sample_rank(double lambda, double eps) {
    if (lambda > 50.0) return (int)std::ceil(lambda + 5.0 * std::sqrt(lambda));  // normal tail, about 3e-7
    double term = std::exp(-lambda), cdf = term;  // P(X <= 0)
    int r = 1;
    while (1.0 - cdf > eps && r < 1 << 20) {
        term *= lambda / r;  // P(X = r)
        cdf += term;
        ++r;
    }
    return r;
}

// The BF16 item table, followed (at the next 256-byte boundary) by 2 n
// floats: bounds on each item row's 2-norm and on its BF16 residual's.
static size_t bf16_table_bytes(const Model &M) { return ((size_t)M.n * round_up(M.k, 32) * 2 + 255) & ~size_t(255); }
static float *bf16_item_norms(Model &M) {
    return reinterpret_cast<float *>(M.Qb.as<unsigned char>() + bf16_table_bytes(M));
}

void ensure_bf16_items(Model &M, bool may_alloc) {
    if (M.bf16_valid) return;
    const int kb = round_up(M.k, 32);
    const size_t need = bf16_table_bytes(M) + (((size_t)M.n * 8 + 255) & ~size_t(255));
    if (M.Qb.bytes < need) {
        if (!may_alloc)
            BMF_FAIL(BMF_E_STATE, "the BF16 item table has no device memory yet: run one BF16 top-K call that may "
                                  "allocate (bmf_topk_bf16, or bmf_topk_dev with precision 1 or 2) first");
        M.Qb.alloc(need);
    }
    const int grid = (int)std::min<int64_t>((M.n * kb + 255) / 256, 8192);
    bf16_table_kernel<<<grid, 256, 0, M.stream>>>(M.Q.as<float>(), M.n, M.k, kb, M.Qb.as<uint16_t>());
    BMF_HIP(hipGetLastError());
    const int ngrid = (int)std::min<int64_t>((M.n + 3) / 4, 8192);  // four rows per 256-thread block
    item_norms_kernel<<<ngrid, 256, 0, M.stream>>>(M.Q.as<float>(), M.n, M.k, bf16_item_norms(M));
    BMF_HIP(hipGetLastError());
    M.bf16_valid = true;
}

TopkPlan topk_plan(const Model &M, int64_t nu, int K, int precision, int Kc) {
    return topk_plan(M.n, M.k, nu, K, precision, Kc);
}

TopkPlan topk_plan(int64_t n, int k, int64_t nu, int K, int precision, int Kc) {
    TopkPlan T;
    T.nu = nu;
    T.K = K;
    T.bf = precision == 1 || precision == 2;
    T.rescore = precision == 1;
    T.Ksel = T.rescore ? topk_candidates(K, Kc) : K;
    {
        const char *e = std::getenv("BMF_TOPK_PRUNE");
        T.prune = (e && e[0] == '0' && e[1] == 0) ? 0 : 1;
    }
    if (K < 1 || T.Ksel > 1008) BMF_FAIL(BMF_E_INVAL, "top-K needs 1 <= K and at most 1008 candidates per user");
    T.kp = round_up(k, 16);
    T.kb = round_up(k, 32);
    T.nu_pad = (nu + TU - 1) / TU * TU;
    const int need = T.Ksel;
    if (need >= n || n <= SAMPLE_MAX) {
        // every item is a candidate
        T.s = 0;
        T.r = 0;
        T.capg = round_up((int)n, 64);
    } else {
        T.s = SAMPLE_MAX;
        T.r = std::min(T.s, sample_rank((double)need * T.s / (double)n, 1e-6));
        // the fraction of the items above the r-th best of s sampled ones is
        // Beta(r, s - r + 1) distributed, about Gamma(r) / (s + 1): r / (s + 1)
        // on average.  The buffer holds three times the mean plus slack, and
        // at least the Gamma(r) quantile of 1 - 1e-9 (Wilson-Hilferty, z = 6)
        // plus slack, so that an overflow (which falls back to the full
        // selection, one wave sweeping every item) stays rarer than about
        // 1e-9 per user when r is small
        const double expect = (double)T.r / (T.s + 1) * (double)n;
        const double c9 = 1.0 / (9.0 * T.r);
        const double wh = 1.0 - c9 + 6.0 * std::sqrt(c9);
        const double tail = (double)T.r * wh * wh * wh / (T.s + 1) * (double)n + 64.0;
        const double want = std::max(3.0 * expect + 128.0, tail);
        T.capg = std::min(CAPG_MAX, round_up((int)std::min(want, (double)CAPG_MAX), 64));
        T.capg = std::max(T.capg, std::min(CAPG_MAX, round_up(need + 64, 64)));
    }
    // item splits for the filter: enough workgroups to fill the chip, and a
    // multiple of 8 (one eighth of the item rows per XCD) where every split
    // still holds at least 256 items
    T.ut = filter_tiles_per_wave(dispatch_kc(T.bf ? T.kb / 32 : T.kp / 16), T.bf);
    const int64_t groups = (T.nu_pad / TU + T.ut - 1) / T.ut;
    int S = (int)std::max<int64_t>(1, (4096 + groups - 1) / std::max<int64_t>(groups, 1));
    if (n >= 8 * 256) S = round_up(S, 8);
    S = (int)std::min<int64_t>(S, std::max<int64_t>(1, n / 256));
    // the filter's lists hold item offsets in 16 bits: at most 65520 items
    // (a multiple of the tile) per split
    S = (int)std::max<int64_t>(S, (n + 65519) / 65520);
    T.per_split = ((n + S - 1) / S + TI - 1) / TI * TI;
    if (T.per_split > 65536) BMF_FAIL(BMF_E_INVAL, "too many items for the top-K filter's splits");
    T.S = (int)std::max<int64_t>(1, (n + T.per_split - 1) / T.per_split);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += (bytes + 255) & ~size_t(255);
        return at;
    };
    T.off_ug = take((size_t)T.nu_pad * T.kp * 4);
    T.off_ugb = take((size_t)T.nu_pad * T.kb * 2);
    T.off_ub = take((size_t)T.nu_pad * 4);
    T.off_thr = take((size_t)T.nu_pad * 4);
    T.off_cnt = take((size_t)T.nu_pad * 4);
    T.off_fail = take((size_t)T.nu_pad * 4);
    T.off_cand = take((size_t)T.nu_pad * std::max(T.capg, T.K) * 8);
    T.off_sel = take((size_t)T.nu_pad * std::max(T.Ksel, T.K) * 8);
    T.total = o;
    return T;
}

void topk_gather(Model &M, const TopkPlan &T, const int32_t *d_users, unsigned char *work, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((T.nu_pad + 3) / 4, 8192);  // four rows per 256-thread block
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
    uint32_t *thr = reinterpret_cast<uint32_t *>(work + T.off_thr);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(work + T.off_cnt);
    uint32_t *fail = reinterpret_cast<uint32_t *>(work + T.off_fail);
    uint64_t *cand = reinterpret_cast<uint64_t *>(work + T.off_cand);
    uint64_t *sel = reinterpret_cast<uint64_t *>(work + T.off_sel);
    if (T.bf) {
        if (!M.bf16_valid) BMF_FAIL(BMF_E_STATE, "BF16 item table not prepared");
        passes_dispatch<true>(T.kb / 32, T, Ug, Ugb, M.Q.as<float>(), M.Qb.as<uint16_t>(), M.bi.as<float>(), M.n, M.k,
                              bf16_item_norms(M), thr, cnt, fail, cand, sel, s);
    } else {
        passes_dispatch<false>(T.kp / 16, T, Ug, Ugb, M.Q.as<float>(), nullptr, M.bi.as<float>(), M.n, M.k, nullptr,
                               thr, cnt, fail, cand, sel, s);
    }
    // every user's best K keys are at sel + row * Ksel
    const int dgrid = (int)std::min<int64_t>((T.nu * T.K + 255) / 256, 8192);
    decode_kernel<<<dgrid, 256, 0, s>>>(sel, T.nu, T.K, T.Ksel, ub, d_items, d_scores);
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
    if (T.bf) ensure_bf16_items(M, true);
    topk_score(M, T, w, d_items, d_scores, M.stream);
}

// ------------------------------------------------ fixed device workspace
// For callers that cannot allocate device memory (work captured into a HIP
// graph, serving loops that must not allocate): the top-K workspace of
// topk_run_fixed lives in this array, TOPK_FIXED_BYTES on every device the
// library runs on, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it names a stand-in, not device
// memory): fixed_workspace() takes its device address once per device with
// hipGetSymbolAddress, and that address is what the kernels get.  Every
// call on one device shares the array; the passes write everything they
// read (the threshold pass clears the candidate counts), so nothing needs
// clearing between calls, and calls that overlap on one device race.
static __device__ __align__(256) unsigned char scratch[TOPK_FIXED_BYTES];

static unsigned char *fixed_workspace(int device) {
    static std::mutex mu;
    static std::vector<unsigned char *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) BMF_FAIL(BMF_E_INVAL, "bad device");
    if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
    if (!addr[device]) {
        void *p = nullptr;
        // the caller has made `device` current (every entry point does)
        BMF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) BMF_FAIL(BMF_E_DEVICE, "no device address for the fixed top-K workspace");
        addr[device] = static_cast<unsigned char *>(p);
    }
    return addr[device];
}

void topk_run_fixed(Model &M, const int32_t *d_users, int64_t nu, int K, int precision, int Kc, int32_t *d_items,
                    float *d_scores) {
    if (M.k > 256) BMF_FAIL(BMF_E_INVAL, "top-K scoring supports k <= 256");
    unsigned char *w = fixed_workspace(M.device);
    if (nu == 0) return;
    const TopkPlan T = topk_plan(M, nu, K, precision, Kc);
    if (T.total > TOPK_FIXED_BYTES)
        BMF_FAIL(BMF_E_NOMEM, "the request needs " + std::to_string(T.total) + " bytes of workspace, more than the " +
                                  std::to_string(TOPK_FIXED_BYTES) + " of the fixed top-K workspace; split it");
    if (T.bf) ensure_bf16_items(M, false);
    topk_gather(M, T, d_users, w, M.stream);
    topk_score(M, T, w, d_items, d_scores, M.stream);
}

}  // namespace bmf
