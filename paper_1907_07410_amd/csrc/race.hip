// Race check of the stratified schedule (Section 3): the b blocks that one
// stratum runs at once must touch disjoint user rows and disjoint item rows,
// since their workgroups update P, bu, Q and bi without locks or atomics.
//
// For every stratum in turn the check walks the records the chosen SGD
// kernel reads for that stratum's blocks, works out the user row and the
// item row each rating updates the way the kernel does, and marks both rows
// in owner arrays with atomicMax of the tag (stratum + 1) * b + column.
// Tags grow from one stratum to the next, so a mark left by an earlier
// stratum is below every tag of the current one.  Of two blocks of one
// stratum that touch the same row, the one that marks it second finds the
// other's tag or a larger one, never its own; a block alone on a row finds
// only its own tag or an older one.  The count of ratings that find a
// foreign tag of their own stratum is therefore zero exactly when the
// stratum's blocks are disjoint.  A record that names a row outside its
// block's range counts as well.

#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"

namespace bmf {
namespace {

constexpr int RACE_WG = 256;

// Mark `row` with `tag`; true when it already held a different tag of the
// current stratum (tags base .. base + b - 1).
__device__ __forceinline__ unsigned mark(unsigned long long *owner, int64_t row, unsigned long long tag,
                                         unsigned long long base) {
    const unsigned long long old = atomicMax(owner + row, tag);
    return old >= base && old != tag ? 1u : 0u;
}

// Partition records (the layout of the global-memory SGD kernels): ui holds
// the user's row within the block row above ibits and the item's column
// within the block column below.  Workgroup w takes column j = w / splits
// of stratum s, paired with block row rows[j] (rows null: (j + s) mod b,
// the schedule the SGD kernels run).
__global__ __launch_bounds__(RACE_WG) void disjoint_recs_kernel(const Rec *__restrict__ recs,
                                                               const int64_t *__restrict__ block_ptr,
                                                               const int32_t *__restrict__ rows, int s, int b,
                                                               int splits, int64_t rb, int64_t cb, int ibits,
                                                               int64_t m,
                                                               int64_t n, unsigned long long base,
                                                               unsigned long long *own_u, unsigned long long *own_i,
                                                               unsigned long long *count) {
    const int j = (int)(blockIdx.x / (unsigned)splits);
    const int part = (int)(blockIdx.x % (unsigned)splits);
    const int64_t br = rows ? rows[j] : (j + s) % b;
    const int64_t blk = br * b + j;
    const int64_t beg = block_ptr[blk], end = block_ptr[blk + 1];
    const uint32_t imask = (1u << ibits) - 1u;
    const unsigned long long tag = base + (unsigned long long)j;
    unsigned bad = 0;
    for (int64_t t = beg + (int64_t)part * RACE_WG + threadIdx.x; t < end; t += (int64_t)splits * RACE_WG) {
        const uint32_t ui = recs[t].ui;
        const int64_t ul = ui >> ibits, il = ui & imask;
        const int64_t u = br * rb + ul, i = (int64_t)j * cb + il;
        if (ul >= rb || u >= m || il >= cb || i >= n) {
            ++bad;
            continue;
        }
        bad += mark(own_u, u, tag, base);
        bad += mark(own_i, i, tag, base);
    }
    if (bad) atomicAdd(count, (unsigned long long)bad);
}

// Step records of the LDS-staged kernel: the item is the LDS row that qa
// addresses (row cb, the dummy, marks an empty position) and the user the
// local row in ulf.  The kernel also writes back its whole item slice,
// which depends on the column alone and so never meets another column's.
__global__ __launch_bounds__(RACE_WG) void disjoint_steps_kernel(const SlotRec *__restrict__ steps,
                                                                const int64_t *__restrict__ blk_step,
                                                                const int32_t *__restrict__ rows, int s, int b,
                                                                int splits, int64_t rb, int64_t cb, uint32_t q0,
                                                                uint32_t row_bytes, int64_t m, int64_t n,
                                                                unsigned long long base, unsigned long long *own_u,
                                                                unsigned long long *own_i,
                                                                unsigned long long *count) {
    const int j = (int)(blockIdx.x / (unsigned)splits);
    const int part = (int)(blockIdx.x % (unsigned)splits);
    const int64_t br = rows ? rows[j] : (j + s) % b;
    const int64_t blk = br * b + j;
    const int64_t beg = blk_step[blk] * PLAN_W, end = blk_step[blk + 1] * PLAN_W;
    const unsigned long long tag = base + (unsigned long long)j;
    unsigned bad = 0;
    for (int64_t t = beg + (int64_t)part * RACE_WG + threadIdx.x; t < end; t += (int64_t)splits * RACE_WG) {
        const SlotRec rec = steps[t];
        if (rec.qa < q0 || (rec.qa - q0) % row_bytes != 0u) {
            ++bad;
            continue;
        }
        const int64_t il = (rec.qa - q0) / row_bytes;
        if (il == cb) continue;  // empty position
        const int64_t ul = rec.ulf & PLAN_UL_MASK;
        const int64_t u = br * rb + ul, i = (int64_t)j * cb + il;
        if (il > cb || ul >= rb || u >= m || i >= n) {
            ++bad;
            continue;
        }
        bad += mark(own_u, u, tag, base);
        bad += mark(own_i, i, tag, base);
    }
    if (bad) atomicAdd(count, (unsigned long long)bad);
}

}  // namespace

bool disjoint_check_env() {
    const char *e = std::getenv("BMF_CHECK_DISJOINT");
    return e && e[0] == '1' && e[1] == 0;
}

int64_t disjoint_check(Model &M, int variant, const int32_t *pairing) {
    if (M.ooc.on) BMF_FAIL(BMF_E_STATE, "the race check needs resident ratings (out-of-core ratings stay on the host)");
    const int b = M.b;
    const Partition &Pt = M.part;
    DevBuf drows, own, cnt;
    if (pairing) {
        const size_t bb = (size_t)b * b;
        for (size_t x = 0; x < bb; ++x)
            if (pairing[x] < 0 || pairing[x] >= b)
                BMF_FAIL(BMF_E_INVAL, "pairing entry " + std::to_string(x) + " is not a block row");
        drows.alloc(bb * 4);
        BMF_HIP(hipMemcpy(drows.p, pairing, bb * 4, hipMemcpyHostToDevice));
    }
    own.alloc((size_t)(M.m + M.n) * 8);
    cnt.alloc(8);
    BMF_HIP(hipMemsetAsync(own.p, 0, own.bytes, M.stream));
    BMF_HIP(hipMemsetAsync(cnt.p, 0, 8, M.stream));
    unsigned long long *own_u = own.as<unsigned long long>(), *own_i = own_u + M.m;
    // enough workgroups per stratum to spread its ratings over the chip
    const int splits = std::max(1, std::min(64, 2048 / b));
    const unsigned grid = (unsigned)b * (unsigned)splits;
    for (int s = 0; s < b; ++s) {
        const int32_t *dr = pairing ? drows.as<int32_t>() + (size_t)s * b : nullptr;
        const unsigned long long base = (unsigned long long)(s + 1) * (unsigned long long)b;
        if (variant == 2) {
            const PlanLds L = plan_lds(M.plan.kp, Pt.cb, M.plan.S, M.plan.CH);
            disjoint_steps_kernel<<<grid, RACE_WG, 0, M.stream>>>(
                M.plan.steps.as<SlotRec>(), M.plan.blk_step.as<int64_t>(), dr, s, b, splits, Pt.rb, Pt.cb,
                (uint32_t)L.q, (uint32_t)L.row_bytes, M.m, M.n, base, own_u, own_i,
                cnt.as<unsigned long long>());
        } else {
            disjoint_recs_kernel<<<grid, RACE_WG, 0, M.stream>>>(Pt.recs.as<Rec>(), Pt.block_ptr.as<int64_t>(), dr, s,
                                                                 b, splits, Pt.rb, Pt.cb, Pt.ibits, M.m, M.n, base,
                                                                 own_u, own_i, cnt.as<unsigned long long>());
        }
        BMF_HIP(hipGetLastError());
    }
    unsigned long long h = 0;
    BMF_HIP(hipMemcpyAsync(&h, cnt.p, 8, hipMemcpyDeviceToHost, M.stream));
    BMF_HIP(hipStreamSynchronize(M.stream));
    return (int64_t)h;
}

}  // namespace bmf
