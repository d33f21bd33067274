// Data-side kernels: factor initialisation, input validation, the global
// mean, and the block partition of the ratings (Section 3's block
// representation; Algorithm 1, steps 1-2; Algorithm 2's row-major visit
// order inside a block).
#include <algorithm>
#include <climits>
#include <cmath>

#include "internal.h"
#include "wave.h"

namespace bmf {

void DevBuf::alloc(size_t n) {
    free_();
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        BMF_FAIL(BMF_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
}

void DevBuf::free_() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// ------------------------------------------------------------- SplitMix64
// Steele, Lea and Flood (OOPSLA 2014), counter form: draw j of the stream
// with seed s is mix(s + (j + 1) * 0x9E3779B97F4A7C15).
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t splitmix64(uint64_t seed, uint64_t j) { return sm64_mix(seed + (j + 1) * 0x9E3779B97F4A7C15ull); }

void schedule(int b, uint64_t seed, int epoch, int mode, int32_t *order) {
    for (int s = 0; s < b; ++s) order[s] = s;
    if (mode == 0) return;
    const uint64_t stream = seed ^ (3ull << 56) ^ ((uint64_t)(uint32_t)epoch << 24);
    for (int t = b - 1; t >= 1; --t) {
        const uint64_t x = splitmix64(stream, (uint64_t)(b - 1 - t));
        const int j = (int)(x % (uint64_t)(t + 1));
        std::swap(order[t], order[j]);
    }
}

// Initial factor entry: (j - 2^23) * 2^-26 with j the top 24 bits of the
// draw, i.e. 0.125 * (2 * j * 2^-24 - 1): exact in FP32.
// Entries t0 .. t1-1 of the row-major table (entry t = row * k + f).
__global__ void init_factors_kernel(float *__restrict__ A, int64_t t0, int64_t t1, uint64_t stream) {
    for (int64_t t = t0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < t1;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = sm64_mix(stream + ((uint64_t)t + 1) * 0x9E3779B97F4A7C15ull);
        const int32_t j = (int32_t)(x >> 40);
        A[t] = (float)(j - 8388608) * 0x1p-26f;
    }
}

void launch_init_factors_rows(float *A, int64_t r0, int64_t r1, int k, uint64_t seed, int tag, hipStream_t s) {
    const int64_t t0 = r0 * (int64_t)k, t1 = r1 * (int64_t)k;
    if (t1 <= t0) return;
    const int grid = (int)std::min<int64_t>((t1 - t0 + 255) / 256, 8192);
    init_factors_kernel<<<grid, 256, 0, s>>>(A, t0, t1, seed ^ ((uint64_t)tag << 56));
    BMF_HIP(hipGetLastError());
}

void launch_init_factors(float *A, int64_t rows, int k, uint64_t seed, int tag, hipStream_t s) {
    launch_init_factors_rows(A, 0, rows, k, seed, tag, s);
}

__global__ void fill_kernel(float *__restrict__ A, int64_t n, float v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        A[t] = v;
}

void launch_fill(float *A, int64_t n, float v, hipStream_t s) {
    if (n == 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_kernel<<<grid, 256, 0, s>>>(A, n, v);
    BMF_HIP(hipGetLastError());
}

// -------------------------------------------------------------- validation
__global__ void validate_kernel(const int32_t *__restrict__ u, const int32_t *__restrict__ i,
                                const float *__restrict__ r, int64_t nnz, int64_t m, int64_t n,
                                unsigned long long *first_bad) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t uu = u[t], ii = i[t];
        const float rr = r[t];
        const bool bad = uu < 0 || (int64_t)uu >= m || ii < 0 || (int64_t)ii >= n || !isfinite(rr);
        if (bad) atomicMin(first_bad, (unsigned long long)t);
    }
}

int64_t validate_coo(const int32_t *u, const int32_t *i, const float *r, int64_t nnz, int64_t m, int64_t n,
                     DevBuf &scratch, hipStream_t s) {
    if (nnz == 0) return -1;
    if (scratch.bytes < 8) scratch.alloc(1 << 16);
    unsigned long long init = ULLONG_MAX, out = 0;
    BMF_HIP(hipMemcpyAsync(scratch.p, &init, 8, hipMemcpyHostToDevice, s));
    const int grid = (int)std::min<int64_t>((nnz + 255) / 256, 4096);
    validate_kernel<<<grid, 256, 0, s>>>(u, i, r, nnz, m, n, scratch.as<unsigned long long>());
    BMF_HIP(hipGetLastError());
    BMF_HIP(hipMemcpyAsync(&out, scratch.p, 8, hipMemcpyDeviceToHost, s));
    BMF_HIP(hipStreamSynchronize(s));
    return out == ULLONG_MAX ? -1 : (int64_t)out;
}

// --------------------------------------------------------- FP64 summation
// Fixed-order sum: thread g of a fixed 256 x 256 grid adds elements g,
// g + 65536, ... sequentially; each workgroup reduces its 256 partials by a
// fixed tree; one workgroup then reduces the 256 workgroup partials.
constexpr int SUM_GRID = 256, SUM_BLOCK = 256;

__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = SUM_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(SUM_BLOCK) void sum_f32_partials_kernel(const float *__restrict__ r, int64_t nnz,
                                                                     double *__restrict__ part) {
    __shared__ double sh[SUM_BLOCK];
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)SUM_BLOCK + threadIdx.x; t < nnz; t += (int64_t)SUM_GRID * SUM_BLOCK)
        acc += (double)r[t];
    const double tot = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SUM_BLOCK) void sum_final_kernel(const double *__restrict__ part, int cnt,
                                                              double *__restrict__ out) {
    __shared__ double sh[SUM_BLOCK];
    double acc = 0.0;
    for (int t = threadIdx.x; t < cnt; t += SUM_BLOCK) acc += part[t];
    const double tot = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) *out = tot;
}

double sum_f32_as_f64(const float *r, int64_t nnz, DevBuf &scratch, hipStream_t s) {
    if (nnz == 0) return 0.0;
    if (scratch.bytes < (SUM_GRID + 1) * sizeof(double)) scratch.alloc(1 << 16);
    double *part = scratch.as<double>();
    sum_f32_partials_kernel<<<SUM_GRID, SUM_BLOCK, 0, s>>>(r, nnz, part);
    BMF_HIP(hipGetLastError());
    sum_final_kernel<<<1, SUM_BLOCK, 0, s>>>(part, SUM_GRID, part + SUM_GRID);
    BMF_HIP(hipGetLastError());
    double out = 0.0;
    BMF_HIP(hipMemcpyAsync(&out, part + SUM_GRID, 8, hipMemcpyDeviceToHost, s));
    BMF_HIP(hipStreamSynchronize(s));
    return out;
}

// --------------------------------------------------------------- partition
// Bucket b_id = (u / rb) * b + (i / cb).  Each rating gets a 64-bit key
// (u_local, i_local, t) packed in (ubits, ibits, tbits) bits; the keys are
// scattered into their buckets (any order) and each bucket is then sorted by
// key, which yields the (u, i, input index) order inside every block.
__global__ void part_hist_kernel(const int32_t *__restrict__ u, const int32_t *__restrict__ i, int64_t nnz,
                                 int64_t rb, int64_t cb, int b, unsigned long long *__restrict__ cnt) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t blk = (u[t] / rb) * b + (i[t] / cb);
        atomicAdd(&cnt[blk], 1ull);
    }
}

// Exclusive scan of nb counts by one workgroup (1024 threads): writes
// block_ptr[0..nb] and a copy of the offsets into the scatter cursors.
__global__ __launch_bounds__(1024) void part_scan_kernel(const unsigned long long *__restrict__ cnt, int64_t nb,
                                                         int64_t *__restrict__ block_ptr,
                                                         unsigned long long *__restrict__ cursor) {
    __shared__ unsigned long long sh[1024];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t q = base + threadIdx.x;
        const unsigned long long v = q < nb ? cnt[q] : 0ull;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            unsigned long long add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0ull;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        const unsigned long long incl = sh[threadIdx.x] + carry;
        if (q < nb) {
            block_ptr[q] = (int64_t)(incl - v);
            cursor[q] = incl - v;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) block_ptr[nb] = (int64_t)carry;
}

__global__ void part_scatter_kernel(const int32_t *__restrict__ u, const int32_t *__restrict__ i, int64_t nnz,
                                    int64_t rb, int64_t cb, int b, int ibits, int tbits,
                                    unsigned long long *__restrict__ cursor, uint64_t *__restrict__ keys) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t uu = u[t], ii = i[t];
        const int64_t br = uu / rb, bc = ii / cb;
        const uint64_t ul = (uint64_t)(uu - br * rb), il = (uint64_t)(ii - bc * cb);
        const unsigned long long pos = atomicAdd(&cursor[br * b + bc], 1ull);
        keys[pos] = (((ul << ibits) | il) << tbits) | (uint64_t)t;
    }
}

// Bitonic sort of one bucket, ascending.  All comparators run ascending:
// stage p compares position x with x ^ (p - 1) (the "flip"), then each
// half-cleaner compares x with x + q.  Pairs whose upper index is at or past
// the bucket size are skipped: those virtual +inf entries never move, so no
// padding is stored.
constexpr int SORT_THREADS = 1024;
constexpr int SORT_LDS = 8192;

template <class Load, class Store>
__device__ __forceinline__ void bitonic_ascending(int64_t size, Load ld, Store st, bool lds) {
    int64_t N = 1;
    while (N < size) N <<= 1;
    for (int64_t p = 2; p <= N; p <<= 1) {
        const int64_t half = p >> 1;
        for (int64_t idx = threadIdx.x; idx < N / 2; idx += SORT_THREADS) {
            const int64_t x = (idx / half) * p + (idx % half);
            const int64_t y = (idx / half) * p + p - 1 - (idx % half);
            if (y < size) {
                const uint64_t a = ld(x), c = ld(y);
                if (a > c) {
                    st(x, c);
                    st(y, a);
                }
            }
        }
        __syncthreads();
        for (int64_t q = half >> 1; q >= 1; q >>= 1) {
            for (int64_t idx = threadIdx.x; idx < N / 2; idx += SORT_THREADS) {
                const int64_t x = (idx / q) * 2 * q + (idx % q);
                const int64_t y = x + q;
                if (y < size) {
                    const uint64_t a = ld(x), c = ld(y);
                    if (a > c) {
                        st(x, c);
                        st(y, a);
                    }
                }
            }
            __syncthreads();
        }
    }
    (void)lds;
}

__global__ __launch_bounds__(SORT_THREADS) void bucket_sort_kernel(uint64_t *__restrict__ keys,
                                                                   const int64_t *__restrict__ block_ptr,
                                                                   int64_t nb) {
    __shared__ uint64_t sh[SORT_LDS];
    for (int64_t q = blockIdx.x; q < nb; q += gridDim.x) {
        const int64_t beg = block_ptr[q], size = block_ptr[q + 1] - beg;
        if (size <= 1) continue;
        uint64_t *g = keys + beg;
        if (size <= SORT_LDS) {
            for (int64_t x = threadIdx.x; x < size; x += SORT_THREADS) sh[x] = g[x];
            __syncthreads();
            bitonic_ascending(
                size, [&](int64_t x) { return sh[x]; }, [&](int64_t x, uint64_t v) { sh[x] = v; }, true);
            for (int64_t x = threadIdx.x; x < size; x += SORT_THREADS) g[x] = sh[x];
            __syncthreads();
        } else {
            bitonic_ascending(
                size, [&](int64_t x) { return __builtin_nontemporal_load(g + x); },
                [&](int64_t x, uint64_t v) { g[x] = v; }, false);
            __syncthreads();
        }
    }
}

__global__ void part_finish_kernel(const uint64_t *__restrict__ keys, int64_t nnz, int tbits, int ibits,
                                   const float *__restrict__ r, Rec *__restrict__ recs, int32_t *__restrict__ perm) {
    const uint64_t tmask = (tbits >= 64) ? ~0ull : ((1ull << tbits) - 1ull);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[p];
        const int64_t t = (int64_t)(key & tmask);
        const uint32_t ui = (uint32_t)(key >> tbits);
        recs[p] = Rec{ui, r[t]};
        perm[p] = (int32_t)t;
    }
    (void)ibits;
}

void block_histogram(const int32_t *u, const int32_t *i, int64_t nnz, int64_t m, int64_t n, int b,
                     std::vector<int64_t> &out, hipStream_t s) {
    const int64_t nb = (int64_t)b * b;
    const int64_t rb = (m + b - 1) / b, cb = (n + b - 1) / b;
    DevBuf cnt;
    cnt.alloc(nb * sizeof(unsigned long long));
    BMF_HIP(hipMemsetAsync(cnt.p, 0, nb * sizeof(unsigned long long), s));
    if (nnz > 0) {
        const int grid = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
        part_hist_kernel<<<grid, 256, 0, s>>>(u, i, nnz, rb, cb, b, cnt.as<unsigned long long>());
        BMF_HIP(hipGetLastError());
    }
    out.resize(nb);
    BMF_HIP(hipMemcpyAsync(out.data(), cnt.p, nb * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BMF_HIP(hipStreamSynchronize(s));
}

static int bits_for(int64_t count) {  // bits to hold values 0..count-1
    int b = 0;
    while (b < 63 && (1ll << b) < count) ++b;
    return b;
}

void build_partition(Partition &out, const int32_t *u, const int32_t *i, const float *r, int64_t nnz, int64_t m,
                     int64_t n, int b, hipStream_t s) {
    Partition P;
    P.nnz = nnz;
    P.rb = (m + b - 1) / b;
    P.cb = (n + b - 1) / b;
    P.ubits = bits_for(P.rb);
    P.ibits = bits_for(P.cb);
    const int tbits = std::max(1, bits_for(nnz));
    if (P.ubits + P.ibits > 32)
        BMF_FAIL(BMF_E_RANGE, "a block of " + std::to_string(P.rb) + " x " + std::to_string(P.cb) +
                                  " cells needs more than 32 bits of local index; use a larger block grid");
    if (P.ubits + P.ibits + tbits > 64) BMF_FAIL(BMF_E_RANGE, "partition key exceeds 64 bits");
    const int64_t nb = (int64_t)b * b;
    P.block_ptr.alloc((nb + 1) * sizeof(int64_t));
    DevBuf cnt, cursor, keys;
    cnt.alloc(nb * sizeof(unsigned long long));
    cursor.alloc(nb * sizeof(unsigned long long));
    BMF_HIP(hipMemsetAsync(cnt.p, 0, nb * sizeof(unsigned long long), s));
    if (nnz > 0) {
        keys.alloc(nnz * sizeof(uint64_t));
        P.recs.alloc(nnz * sizeof(Rec));
        P.perm.alloc(nnz * sizeof(int32_t));
        const int grid = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
        part_hist_kernel<<<grid, 256, 0, s>>>(u, i, nnz, P.rb, P.cb, b, cnt.as<unsigned long long>());
        BMF_HIP(hipGetLastError());
    }
    part_scan_kernel<<<1, 1024, 0, s>>>(cnt.as<unsigned long long>(), nb, P.block_ptr.as<int64_t>(),
                                        cursor.as<unsigned long long>());
    BMF_HIP(hipGetLastError());
    if (nnz > 0) {
        const int grid = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
        part_scatter_kernel<<<grid, 256, 0, s>>>(u, i, nnz, P.rb, P.cb, b, P.ibits, tbits,
                                                 cursor.as<unsigned long long>(), keys.as<uint64_t>());
        BMF_HIP(hipGetLastError());
        const int sgrid = (int)std::min<int64_t>(nb, 2048);
        bucket_sort_kernel<<<sgrid, SORT_THREADS, 0, s>>>(keys.as<uint64_t>(), P.block_ptr.as<int64_t>(), nb);
        BMF_HIP(hipGetLastError());
        part_finish_kernel<<<grid, 256, 0, s>>>(keys.as<uint64_t>(), nnz, tbits, P.ibits, r, P.recs.as<Rec>(),
                                                P.perm.as<int32_t>());
        BMF_HIP(hipGetLastError());
    }
    P.h_block_ptr.resize(nb + 1);
    BMF_HIP(hipMemcpyAsync(P.h_block_ptr.data(), P.block_ptr.p, (nb + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                           s));
    BMF_HIP(hipStreamSynchronize(s));
    std::swap(out.nnz, P.nnz);
    std::swap(out.rb, P.rb);
    std::swap(out.cb, P.cb);
    std::swap(out.ubits, P.ubits);
    std::swap(out.ibits, P.ibits);
    out.recs.swap(P.recs);
    out.perm.swap(P.perm);
    out.block_ptr.swap(P.block_ptr);
    out.h_block_ptr.swap(P.h_block_ptr);
}

}  // namespace bmf
