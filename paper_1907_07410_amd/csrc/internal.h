// Internal declarations shared by the libbmf translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bmf.h"
#include "plan.h"

namespace bmf {

// ---------------------------------------------------------------- errors
struct Error {
    bmf_status code;
    std::string msg;
};

#define BMF_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::bmf::Error{BMF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define BMF_FAIL(code, msg) throw ::bmf::Error{(code), (msg)}

// ---------------------------------------------------------- hyper-params
// {alpha_p, beta_p, alpha_q, beta_q, alpha_bu, beta_bu, alpha_bi, beta_bi}
struct HP {
    float a_p, b_p, a_q, b_q, a_bu, b_bu, a_bi, b_bi;
};

// A rating inside a block: local row (u - br*rb) and column (i - bc*cb)
// packed as (row << ibits) | col, and the value.
struct Rec {
    uint32_t ui;
    float r;
};

struct BatchProblem {
    const SlotRec *steps;
    const int64_t *blk_step;
    float *P, *Q, *bu, *bi;
    int64_t n, rb, cb;
    float mu;
    int b, S, CH;
};

struct BatchItem {
    int32_t p, t, s, j;
};

// Device buffer owned by a context.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void alloc(size_t n);
    void free_();
    template <class T> T *as() const { return static_cast<T *>(p); }
    ~DevBuf() { free_(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    void swap(DevBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
};

// Pinned host buffer (hipHostMalloc), for copies that overlap kernels.
struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void alloc(size_t n);
    void free_();
    template <class T> T *as() const { return static_cast<T *>(p); }
    ~PinnedBuf() { free_(); }
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    void swap(PinnedBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
};

// Partition of a rating set on the device.
struct Partition {
    int64_t nnz = 0;
    int64_t rb = 1, cb = 1;
    int ibits = 0, ubits = 0;
    DevBuf recs;       // Rec[nnz], processing order
    DevBuf perm;       // int32[nnz], position -> input index
    DevBuf block_ptr;  // int64[b*b + 1]
    std::vector<int64_t> h_block_ptr;
};

// Execution plan of the LDS-staged SGD kernel (see plan.hip).
struct Plan {
    bool built = false;  // build_plan has run (ok says whether it applies)
    bool ok = false;
    int kp = 0, S = 0, CH = PLAN_CH;
    int64_t total_steps = 0;
    DevBuf steps;     // SlotRec[total_steps * PLAN_W]
    DevBuf blk_step;  // int64[b*b + 1], step offsets per block
    std::vector<int64_t> h_blk_step;
    void swap(Plan &o) {
        std::swap(built, o.built);
        std::swap(ok, o.ok);
        std::swap(kp, o.kp);
        std::swap(S, o.S);
        std::swap(CH, o.CH);
        std::swap(total_steps, o.total_steps);
        steps.swap(o.steps);
        blk_step.swap(o.blk_step);
        h_blk_step.swap(o.h_blk_step);
    }
};

// Out-of-core training data: the stratum work (planned steps or records)
// in pinned host memory, stratum after stratum, each followed by its block
// table (b + 1 unit offsets, by position); OOC_BUFS device buffers take
// turns receiving strata on the copy stream while earlier ones run.
constexpr int OOC_BUFS = 3;
// Strata per ring buffer: at most OOC_GROUP, and as many as fit in
// OOC_SLOT_BYTES (at least one).
constexpr int OOC_GROUP = 8;
constexpr size_t OOC_SLOT_BYTES = size_t(64) << 20;
struct OutOfCore {
    bool on = false;
    int variant = 1;        // 1: records for the reference kernels, 2: planned steps
    size_t unit = 0;        // bytes per unit (one record, or one step of PLAN_W slot records)
    int group = 1;          // strata per ring buffer (one copy, one wait each way per group)
    std::vector<int64_t> s_off;    // b + 1 byte offsets of the strata in `data`
    std::vector<int64_t> s_units;  // units of each stratum (its table follows them)
    PinnedBuf data;                // stratum-major units and tables
    PinnedBuf cu, ci, cr;        // the training COO as given, for RMSE and loss
    std::vector<int32_t> perm;   // processing position -> input index
    DevBuf stage[OOC_BUFS];
    hipStream_t copy = nullptr;
    hipEvent_t copied[OOC_BUFS] = {}, used[OOC_BUFS] = {};
    bool used_valid[OOC_BUFS] = {};
    int64_t ring = 0;  // groups sent so far: the next one goes to buffer ring % OOC_BUFS
    void release();
    ~OutOfCore() { release(); }
};

// An epoch's stratum launches captured once as a HIP graph and replayed
// while nothing they depend on changes (the key: kernel, data and factor
// pointers, sizes, mu, the hyper-parameters and the stratum order).  For
// grids of many small blocks, where launching dominates.
struct EpochGraph {
    bool on = false;
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t captures = 0;
    void reset();
    ~EpochGraph() { reset(); }
};

// --------------------------------------------------------------- context
struct Model {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    int64_t m = 0, n = 0;
    int k = 0, b = 0;
    uint64_t seed = 1001, order_seed = 2001;
    int order_mode = 0, mu_mode = 0, sgd_kernel = 0, waves = 8;
    bool out_of_core = false;  // the next load keeps the ratings in host memory
    DevBuf P, Q, bu, bi;
    double mu = 0.0;
    // training data
    bool loaded = false;
    DevBuf cu, ci, cr;  // training COO as given (int32, int32, f32)
    Partition part;
    Plan plan;
    OutOfCore ooc;
    EpochGraph egraph;
    int32_t epoch = 0;
    // bf16 copies for scoring
    DevBuf Pb, Qb;
    bool bf16_valid = false;
    // timing of SGD launches: event pairs still pending, and spare events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> spare_events;
    double sgd_ms = 0.0;
    int64_t sgd_launches = 0;
    // scratch for reductions / top-K
    DevBuf red;
    DevBuf scratch;
};

}  // namespace bmf

struct bmf_ctx {
    bmf::Model M;
    bool poisoned = false;
    std::string err;
};

namespace bmf {

// ---------------------------------------------------------------- random
uint64_t splitmix64(uint64_t seed, uint64_t j);
void schedule(int b, uint64_t seed, int epoch, int mode, int32_t *order);

// --------------------------------------------------------------- kernels
// all launchers enqueue on `s` and throw Error on launch failure
void launch_init_factors(float *A, int64_t rows, int k, uint64_t seed, int tag, hipStream_t s);
// rows r0 .. r1-1 only (the entries a table of r1 rows would hold there)
void launch_init_factors_rows(float *A, int64_t r0, int64_t r1, int k, uint64_t seed, int tag, hipStream_t s);
void launch_fill(float *A, int64_t n, float v, hipStream_t s);

// Validate COO: returns first bad index or -1 (synchronises).
int64_t validate_coo(const int32_t *u, const int32_t *i, const float *r, int64_t nnz, int64_t m,
                     int64_t n, DevBuf &scratch, hipStream_t s);
// FP64 sum of r[0..nnz) in a fixed order (synchronises).
double sum_f32_as_f64(const float *r, int64_t nnz, DevBuf &scratch, hipStream_t s);
// Ratings per block of a b x b grid, block id row * b + column (synchronises).
void block_histogram(const int32_t *u, const int32_t *i, int64_t nnz, int64_t m, int64_t n, int b,
                     std::vector<int64_t> &out, hipStream_t s);
// Build a partition (synchronises).
void build_partition(Partition &out, const int32_t *u, const int32_t *i, const float *r, int64_t nnz,
                     int64_t m, int64_t n, int b, hipStream_t s);

// Plans: LDS row length for k factors (16 lanes x 1, 2, 4 or 8 floats; 0
// when k > 128), user slots that fit next to a cb-row item slice, one
// block's schedule (host; returns the step count, appends PLAN_W records
// per step), and the whole partition's plan (leaves out.ok false when the
// planned kernel does not apply).
int plan_kp(int k);
int plan_slots(int kp, int64_t cb, int CH, int max_lds);
int64_t plan_block(const uint32_t *ui, int64_t n, int ibits, int cb, int S, int CH, std::vector<PlanEntry> &out);
// Length of the longest chain of ratings (in processing order) in which each
// rating shares its user or its item with the one before it.
int64_t chain_depth(const int32_t *u, const int32_t *i, int64_t n);
void build_plan(Plan &out, const Partition &part, int b, int k, int max_lds, hipStream_t s);
// The host part of build_plan: plan the records (host, processing order)
// into `flat`; false (out.ok false) when the planned kernel does not apply.
bool plan_host(Plan &out, const Rec *recs, const std::vector<int64_t> &block_ptr, int ibits, int ubits, int64_t cb,
               int b, int k, int max_lds, std::vector<SlotRec> &flat);
// The planned kernel's fixed cost per workgroup (staging a full LDS buffer)
// outweighs its gain on blocks of a few ratings: automatic selection takes
// it only when the blocks hold at least PLAN_MIN_MEAN ratings on average.
constexpr int PLAN_MIN_MEAN = 8;
inline bool plan_pays(int64_t nnz, int b) { return nnz >= (int64_t)PLAN_MIN_MEAN * b * b; }
// Build M's plan now if no load or earlier epoch has (synchronises).
void ensure_plan(Model &M);

// SGD: run one epoch of strata in `order`.
void sgd_epoch(Model &M, const int32_t *order, const HP &hp);
// The SGD kernel an epoch of M would run (1 or 2; builds the plan when it
// picks 2).
int sgd_variant(Model &M);
// Race check of the resident ratings' strata for SGD kernel `variant`:
// stratum s pairs column j with block row pairing[s * b + j] (host array;
// nullptr: (j + s) mod b).  Returns the count of ratings whose user or item
// row another block of their stratum also touches, or that name a row
// outside their block (synchronises).
int64_t disjoint_check(Model &M, int variant, const int32_t *pairing);
// BMF_CHECK_DISJOINT=1 in the environment: every resident epoch runs the
// race check first.
bool disjoint_check_env();
// Where one stratum's work is: records (reference kernels) or steps
// (planned kernel), and its block table, indexed br * row_stride + j.
struct StratumData {
    const void *data;
    const int64_t *table;
    int64_t row_stride;
};
// Launch stratum s with SGD kernel `variant` (1 or 2).
void launch_stratum(Model &M, int s, const HP &hp, int variant, const StratumData &D);
// Out-of-core: load host COO (validates, partitions and plans on the host),
// run an epoch's strata with the copies overlapped, and the training
// squared-residual sum (with the loss terms when loss_hp) in chunks.
void ooc_load(Model &M, const int32_t *u, const int32_t *i, const float *r, int64_t nnz);
void ooc_epoch(Model &M, const int32_t *order, const HP &hp, int variant);
double ooc_sq_sum(Model &M, const HP *loss_hp);
// The device's per-workgroup LDS maximum.
int sgd_max_lds(int device);
// One launch running the blocks items[0 .. count) of several problems
// (one position of each) with the planned kernel.
void sgd_positions_launch(int k, int nw, const BatchProblem *d_probs, const BatchItem *d_items, int64_t count,
                          const HP &hp, size_t lds, hipStream_t s);

// Evaluation: sum of squared residuals (FP64) over COO, optionally with
// the regularisation terms (loss). Synchronises.
double sq_residual_sum(const Model &M, const int32_t *u, const int32_t *i, const float *r, int64_t cnt,
                       const HP *loss_hp, DevBuf &scratch);

// Top-K.  A plan fixes the threshold sample, the split of the item range
// and the workspace layout (user vectors FP32/BF16, per-user offsets
// mu + bu, thresholds, candidate buffers and lists); gather fills the user
// vectors from P, score runs threshold, filter, finish, the full-selection
// pass for users that need it, rescore and decode.  topk_run does both on
// M.stream.
struct TopkPlan {
    int64_t nu = 0, nu_pad = 0;
    int K = 0, Ksel = 0, kp = 0, kb = 0;
    bool bf = false;
    // BF16: rescore the candidates in FP32 (precision 1); without it
    // (precision 2) the answer is the BF16 top K with its BF16 scores
    bool rescore = false;
    // BF16: drop candidates that provably cannot reach the FP32 top K before
    // rescoring (on unless BMF_TOPK_PRUNE=0 is in the environment)
    int prune = 1;
    // threshold sample: s items, threshold = the r-th best sampled score
    // (r = 0: no threshold); candidate buffers of capg keys per user;
    // the filter splits the item range into S pieces of per_split items
    int s = 0, r = 0, capg = 0, S = 1;
    // user tiles (16 users each) per filter wave
    int ut = 1;
    int64_t per_split = 0;
    size_t off_ug = 0, off_ugb = 0, off_ub = 0, off_thr = 0, off_cnt = 0, off_fail = 0, off_cand = 0, off_sel = 0,
           total = 0;
};
TopkPlan topk_plan(const Model &M, int64_t nu, int K, int precision, int Kc);
// The same plan from the item count and factor count alone (host only).
TopkPlan topk_plan(int64_t n, int k, int64_t nu, int K, int precision, int Kc);
// BF16 candidates per user for a top-K request: Kc when given (at least K),
// else K + max(16, K / 2).
inline int topk_candidates(int K, int Kc) { return Kc > 0 ? (Kc > K ? Kc : K) : K + (K / 2 > 16 ? K / 2 : 16); }
void topk_gather(Model &M, const TopkPlan &T, const int32_t *d_users, unsigned char *work, hipStream_t s);
void topk_score(Model &M, const TopkPlan &T, unsigned char *work, int32_t *d_items, float *d_scores, hipStream_t s);
void topk_run(Model &M, const int32_t *d_users, int64_t nu, int K, int precision, int Kc,
              int32_t *d_items, float *d_scores);
// topk_run with its workspace in a fixed device array of TOPK_FIXED_BYTES
// (no device allocation: BMF_E_NOMEM when the request needs more; BF16
// needs the item table's memory from an earlier BF16 call, BMF_E_STATE
// otherwise).
constexpr size_t TOPK_FIXED_BYTES = size_t(64) << 20;
void topk_run_fixed(Model &M, const int32_t *d_users, int64_t nu, int K, int precision, int Kc,
                    int32_t *d_items, float *d_scores);
void foldin_run(Model &M, const int32_t *d_items, const float *d_r, int nr, int passes, const HP &hp,
                float *d_p, float *d_bu);
void foldin_launch(Model &M, const int32_t *d_items, const float *d_r, const int64_t *d_off, int64_t nreq,
                   int max_cnt, int passes, const HP &hp, float *d_p, int64_t p_stride, float *d_bu, hipStream_t s);
// Turn folded-in users (p rows written with stride kp, biases bu_f) into
// scoring rows: zero the padding, BF16 copy, offset mu + bu.
void foldin_rows(const float *bu_f, int64_t nreq, float mu, int k, int kp, int kb, float *Ug, uint16_t *Ugb,
                 float *ub, hipStream_t s);
// The BF16 copy of Q for scoring, made after the factors last changed;
// may_alloc false refuses (BMF_E_STATE) where its memory is missing.
void ensure_bf16_items(Model &M, bool may_alloc);

// Timing: take an event (from the spare list or new), and fold completed
// pending pairs into sgd_ms (all of them, waiting, when `wait`).
hipEvent_t take_event(Model &M);
void harvest_timing(Model &M, bool wait);

// Diagnostics: the three wavefront sums of 64 values (xor butterfly, DPP
// butterfly, 16-lane row sums) on the device.
void debug_wave_sum(const float *d_in, float *d_out, hipStream_t s);
// The planned kernel's dependent-step floor: one wavefront, `chunks` chunks
// of PLAN_CH steps whose every step depends on the one before; d_out
// receives 8 (16 F + 4) floats (k <= 128).
void chain_floor(int k, int chunks, float *d_out, hipStream_t s);

}  // namespace bmf
