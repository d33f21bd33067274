// Step plans of the LDS-staged SGD kernel: records, LDS layout, host
// scheduler (plan.hip) and the kernel's use of them (sgd.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace bmf {

// Plans of the LDS-staged SGD kernel (plan.hip).  The scheduler fills PLAN_W
// positions per step with a rating index (-1 when empty) and the LDS slot of
// its user.
struct PlanEntry {
    int32_t x;
    int32_t slot;
};
// Device record of one position (16 bytes): LDS byte offsets (from the
// start of the kernel's dynamic LDS) of the item row and of the user slot
// row (each row holds kp factors, then the bias), the rating, and the
// user's local row | FIRST | LAST.  FIRST: the user's first rating in the
// block (its row is loaded into the slot before the step's chunk); LAST:
// its final one (the slot is written back after the step's chunk).  Empty
// positions point at the dummy item row and dummy slot, with ulf = 0.
struct SlotRec {
    uint32_t qa;
    float r;
    uint32_t ua;
    uint32_t ulf;
};
constexpr int PLAN_W = 4;            // ratings per step (16-lane groups of one wavefront)
#ifndef BMF_PLAN_CH
#define BMF_PLAN_CH 16
#endif
constexpr int PLAN_CH = BMF_PLAN_CH;  // steps per chunk
constexpr int PLAN_MAX_HELPERS = 7;  // helper wavefronts per workgroup, at most
// The planned kernels use a static LDS buffer of this size (all of a gfx950
// CU's LDS; a workgroup per CU), so LDS addresses fold into instructions.
constexpr int PLAN_LDS_BYTES = 160 * 1024;
constexpr int PLAN_MAX_SLOTS = 4095;
constexpr int PLAN_MIN_SLOTS = 8;
constexpr uint32_t PLAN_FIRST = 1u << 30, PLAN_LAST = 1u << 31, PLAN_UL_MASK = (1u << 30) - 1u;

// LDS layout of the planned kernel: the item slice (cb + 1 rows, the last a
// dummy for empty positions), three chunks of records, per-helper
// compaction lists, and S + 1 user slots (slot S the dummy).  A row is kp
// factors followed by the bias, padded to kp + 4 floats.
struct PlanLds {
    size_t q, rec, scr, u, total;
    int row_bytes;
};
__host__ __device__ inline PlanLds plan_lds(int kp, int64_t cb, int S, int CH) {
    PlanLds L;
    L.row_bytes = (kp + 4) * 4;
    size_t o = 0;
    L.q = o;
    o += (size_t)(cb + 1) * L.row_bytes;
    L.rec = o;
    o += (size_t)3 * CH * PLAN_W * sizeof(SlotRec);
    L.scr = o;
    o += (size_t)PLAN_MAX_HELPERS * 64 * 8;
    L.u = o;
    o += (size_t)(S + 1) * L.row_bytes;
    L.total = o;
    return L;
}

}  // namespace bmf
