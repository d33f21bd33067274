/*
 * bmf.h -- C ABI of libbmf: block-based biased-SVD matrix factorisation
 * trained by stratified block-parallel SGD on one AMD MI355X (gfx950).
 *
 * Method: Bhavana, Kumar, Padmanabhan, "Block based Singular Value
 * Decomposition approach to matrix factorization for recommender systems"
 * (arXiv 1907.07410).  X is an m x n rating matrix, m users (rows) and n
 * items (columns) (Section 3, Algorithm 1's inputs); U = P (m x k) and
 * V = Q (n x k) are the latent factors, bu (m) and bi (n) the biases
 * (Algorithm 1; Eq 3); the prediction is mu + bu_u + bi_i + p_u . q_i.
 *
 * Conventions for every call:
 *  - Every call returns bmf_status: 0 on success, a negative code on error.
 *    No C++ exception crosses this boundary.  bmf_last_error(ctx) returns a
 *    message for the last failed call on ctx (bmf_last_error(NULL): the last
 *    failed create on this thread).
 *  - Validation errors (BMF_E_INVAL, BMF_E_RANGE, BMF_E_STATE, BMF_E_NOMEM)
 *    leave the context exactly as it was.  BMF_E_DEVICE (a HIP runtime error)
 *    poisons the context: afterwards only bmf_get_factors, bmf_last_error
 *    and bmf_destroy are accepted.
 *  - Host pointers (plain names) are read or written before the call
 *    returns; the library never keeps them.  Output buffers are allocated by
 *    the caller with the documented sizes.  "_dev" calls take device
 *    pointers on the context's device and only enqueue work on the
 *    context's stream (BMF_OPT_STREAM): they return before the GPU is done.
 *  - The context owns all device memory it allocates.  A context is used by
 *    one host thread at a time; distinct contexts are independent.
 *  - Factor tables are FP32, row-major: P[u*k + f], Q[i*k + f].  Reductions
 *    that report RMSE or loss accumulate in FP64.
 */
#ifndef BMF_H
#define BMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmf_ctx bmf_ctx;
typedef struct bmf_batch bmf_batch;
typedef struct bmf_server bmf_server;

typedef enum {
    BMF_OK = 0,
    BMF_E_INVAL = -1,  /* bad argument (null pointer, size <= 0, bad option) */
    BMF_E_RANGE = -2,  /* an index or value outside its domain */
    BMF_E_STATE = -3,  /* call not allowed in the current state */
    BMF_E_NOMEM = -4,  /* device or host allocation failed / budget exceeded */
    BMF_E_DEVICE = -5  /* HIP runtime error; the context is poisoned */
} bmf_status;

typedef enum {
    /* seed of the initial factors, default 1001.  Setting it re-draws P and
     * Q (Algorithm 1 initialises them "with random values"): entry (row, f)
     * of tensor T (1 = P, 2 = Q) is 0.125 * (2 * (x >> 40) * 2^-24 - 1),
     * x = SplitMix64 draw number row*k + f of the stream seed ^ (T << 56);
     * biases start at 0. */
    BMF_OPT_SEED = 0,
    /* seed of the per-epoch stratum order (mode 1), default 2001 */
    BMF_OPT_ORDER_SEED = 1,
    /* 0: strata 0, 1, ..., b-1 every epoch (Section 3: the diagonal first,
     *    then the blocks below it, columns wrapping);
     * 1: a Fisher-Yates shuffle of 0..b-1 per epoch e drawn from the
     *    SplitMix64 stream order_seed ^ (3 << 56) ^ (e << 24)
     *    (for t = b-1..1: j = draw(b-1-t) mod (t+1), swap t and j).
     * Default 0. */
    BMF_OPT_STRATUM_ORDER = 2,
    /* 0: mu = FP64 mean of the training ratings (default);
     * 1: mu = 0 (Eq 3 taken literally). Takes effect at the next load. */
    BMF_OPT_MU_MODE = 3,
    /* hipStream_t (cast to int64) on which all work is enqueued; 0 = the
     * context's own stream. */
    BMF_OPT_STREAM = 4,
    /* SGD kernel: 0 = automatic (2 when the plan applies and the blocks hold
     * at least 8 ratings on average, else 1), 1 = global-memory reference
     * kernel running each block's ratings in (u, i, t) order, 2 = LDS-staged
     * planned kernel: the block's item slice and its active users' rows in
     * LDS, four independent ratings per step (a list schedule that reorders
     * only ratings sharing neither user nor item, built on the host at load
     * when an epoch will use it, else at the first epoch that does).  For
     * k <= 128, 1 and 2 give identical bits; 2 needs k <= 128 and an item
     * slice that leaves room in LDS for at least 8 user slots (BMF_E_STATE
     * otherwise). */
    BMF_OPT_SGD_KERNEL = 5,
    /* waves per workgroup of the LDS-staged SGD kernel: 4 or 8 (one wave
     * runs the update steps, the others stage data); default 8.  On a
     * batch, 0 lets the autotuner choose.  Does not change results. */
    BMF_OPT_WAVES_PER_BLOCK = 6,
    /* 1: the next load keeps the ratings in pinned host memory (out of core,
     * Section 6's unbounded block count): partition and step plans are made
     * on the host, each stratum's work is laid out contiguously, and an epoch
     * copies groups of strata (up to 8, at most 64 MiB when a stratum is
     * smaller, else one) in the epoch's order into a ring of three device
     * buffers on a copy stream while earlier groups run.  Device memory then
     * holds the factor tables and three such groups.  An out-of-core epoch
     * call waits on the host until a ring buffer is free before it queues the
     * copy into it, so it returns when its last group is queued (about two
     * groups before the epoch ends), and it cannot be captured into a HIP
     * graph.  The kernels, and so the results, are
     * those of a resident load with the same SGD kernel; mu is summed on the
     * host in input order.  Such a load takes host arrays only
     * (bmf_load_ratings), fixes the SGD kernel (set BMF_OPT_SGD_KERNEL before
     * it), and bmf_add_ratings refuses the context.  0 (default): resident. */
    BMF_OPT_OUT_OF_CORE = 7,
    /* The epoch counter: the index of the next epoch (0 <= value < 2^31),
     * which picks its stratum order in mode 1 (BMF_OPT_STRATUM_ORDER).  With
     * factors saved by bmf_get_factors after e epochs and restored by
     * bmf_set_factors into a context loaded with the same ratings, setting
     * it to e makes the following epochs those of the uninterrupted run
     * (Algorithm 1's loop resumed at iteration e). */
    BMF_OPT_EPOCH = 8,
    /* 1: resident epochs capture their b stratum launches as a HIP graph and
     * replay it while the kernel, data, factor tables, mu, hyper-parameters
     * and stratum order stay the same (identical results, fewer launch
     * costs: for grids of many small blocks, such as Section 5's 3072 x 3072).
     * A change of any of them captures again; with a seeded stratum order
     * (mode 1) that is every epoch, so use it with mode 0.  Out-of-core
     * epochs ignore it.  0 (default): direct launches. */
    BMF_OPT_EPOCH_GRAPH = 9
} bmf_option;

/* ------------------------------------------------------------- lifetime */

/* Create a model for m users, n items, k latent factors and a b x b block
 * grid (Algorithm 1, steps 1-2; Section 3's block representation).  Blocks
 * have rb = ceil(m/b) rows and cb = ceil(n/b) columns; the last block row or
 * column may be short or empty.  Allocates P, Q, bu, bi on the current HIP
 * device and draws P and Q as described under BMF_OPT_SEED.
 * Errors: BMF_E_INVAL if out == NULL or m, n, k, b < 1 or k > 1024;
 * BMF_E_NOMEM; BMF_E_DEVICE. */
bmf_status bmf_create(int64_t m, int64_t n, int32_t k, int32_t b, bmf_ctx **out);

/* Set an option (bmf_option).  Errors: BMF_E_INVAL for an unknown key or a
 * value outside the documented set. */
bmf_status bmf_set_option(bmf_ctx *c, int32_t key, int64_t value);

/* Release everything the context owns.  c may be NULL. */
void bmf_destroy(bmf_ctx *c);

/* Message for the last failed call on c (c == NULL: last failed create on
 * this thread).  Valid until the next call on c. */
const char *bmf_last_error(const bmf_ctx *c);

/* Wait for all work enqueued on the context's stream. */
bmf_status bmf_synchronize(bmf_ctx *c);

/* ------------------------------------------------------------- training */

/* Load the training ratings as COO triples (u[t], i[t], r[t]), t < nnz,
 * copied from host memory.  Every triple is an observation (ratings <= 0
 * included); duplicates are separate observations.  Checks 0 <= u < m,
 * 0 <= i < n and finite r (BMF_E_RANGE names the first bad index), computes
 * mu, and partitions the ratings into the b x b blocks on the device: block
 * (u / rb, i / cb), visited inside a block in (u, i, t) order (Algorithm 2's
 * row and column loops); then builds the LDS kernel's per-block step plan
 * on the host (the partition is copied back for it).  Replaces previously
 * loaded ratings; keeps the factors.  nnz may be 0 (then u, i, r may be
 * NULL).
 * Errors: BMF_E_INVAL, BMF_E_RANGE (also when a block's local (row, column)
 * needs more than 32 bits: use a larger b), BMF_E_NOMEM, BMF_E_DEVICE. */
bmf_status bmf_load_ratings(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r,
                            int64_t nnz);

/* Same with device pointers (int32 u, int32 i, float r on the context's
 * device).  Synchronises the stream before returning. */
bmf_status bmf_load_ratings_dev(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r,
                                int64_t nnz);

/* One epoch (one iteration of Algorithm 1's loop): the b strata in this
 * epoch's order (BMF_OPT_STRATUM_ORDER); within a stratum s the b blocks
 * ((j + s) mod b, j), which share no user and no item, run concurrently;
 * every training rating is visited exactly once (Section 3).  Per rating
 * (Eqs 10-13 with one residual taken before any update):
 *   err  = r - mu - bu_u - bi_i - p_u . q_i
 *   bu_u += lr (err - reg bu_u);  bi_i += lr (err - reg bi_i)
 *   p_u  += lr (err q_i - reg p_u);  q_i += lr (err p_u - reg q_i)
 * with p_u and q_i on the right-hand sides taken before the update.
 * Enqueued on the context's stream; returns without waiting.
 * Errors: BMF_E_STATE before a load (and, with BMF_CHECK_DISJOINT=1, when
 * the race check of bmf_check_disjoint finds a shared row); BMF_E_DEVICE. */
bmf_status bmf_epoch(bmf_ctx *c, float lr, float reg);

/* Same with the four (alpha, beta) pairs of Eqs 10-13 given by name:
 * hp = {alpha_p, beta_p, alpha_q, beta_q, alpha_bu, beta_bu, alpha_bi,
 * beta_bi} (user latent, item latent, user bias, item bias). */
bmf_status bmf_epoch_hp(bmf_ctx *c, const float hp[8]);

/* Number of epochs run so far (the next epoch's index). */
bmf_status bmf_epoch_count(const bmf_ctx *c, int32_t *out);

/* What the next epoch runs (Section 3's blocks, Eqs 10-13): *kernel = 2 for
 * the LDS-staged planned kernel, 1 for the 16-lane reference kernel, 3 for
 * the 64-lane reference kernel (k > 128), 0 when kernel 2 is forced but
 * does not apply (the epoch would fail); *steps = the plan's total dependent
 * steps (four ratings each), *slots = LDS user slots per block and
 * block_steps[b*b] = each block's steps (block id row * b + column) when the
 * planned kernel runs, else zeros.  May build the plan (host, synchronises).
 * Any output may be NULL.  Errors: BMF_E_STATE (no ratings loaded). */
bmf_status bmf_plan_info(bmf_ctx *c, int32_t *kernel, int64_t *steps, int32_t *slots, int64_t *block_steps);

/* Incremental data (Section 6: new ratings become new blocks that are
 * factorised on their own, then the factors converge together on all the
 * data).  Grows the model to m_new >= m users and n_new >= n items: learned
 * rows are kept, new rows of P and Q get the seeded initial values a model
 * created at the new size holds there, new biases are 0; the block geometry
 * follows the new sizes.  Then runs epochs_new epochs (pairs hp, as
 * bmf_epoch_hp) over the new ratings u/i/r (host arrays of nnz entries, ids
 * below m_new / n_new) alone, partitioned on the grown b x b grid, starting
 * from the current factors, and finally makes the union (the loaded ratings
 * followed by the new ones) the training set, so that bmf_epoch / bmf_fit
 * continue on all ratings.  mu becomes the union's mean (BMF_OPT_MU_MODE 0)
 * or stays 0 (mode 1) and is used in both phases.  Each phase epoch counts in
 * bmf_epoch_count.  Not to be called while a server uses the context.
 * Errors (nothing changed): BMF_E_INVAL (a size shrinks or reaches 2^31, hp
 * NULL or not finite, epochs_new < 0, nnz < 0, null arrays, the union
 * reaches 2^31 ratings), BMF_E_RANGE (a new rating outside m_new x n_new or
 * not finite); BMF_E_NOMEM / BMF_E_DEVICE afterwards. */
bmf_status bmf_add_ratings(bmf_ctx *c, int64_t m_new, int64_t n_new, const int32_t *u, const int32_t *i,
                           const float *r, int64_t nnz, const float hp[8], int32_t epochs_new);

/* Algorithm 1's loop: epochs with the pairs hp (as bmf_epoch_hp) until the
 * training RMSE improves by less than delta over the previous epoch (the
 * first epoch compares with the RMSE before it), at most max_epochs; an
 * epoch whose RMSE is not a number (diverged training) also ends the loop.
 * *epochs_out receives the epochs run, *rmse_out the final training RMSE
 * (either may be NULL).  Synchronises after every epoch (the RMSE).
 * Errors: BMF_E_INVAL (hp NULL or not finite, max_epochs < 0, delta not
 * finite), BMF_E_STATE (no ratings), BMF_E_DEVICE. */
bmf_status bmf_fit(bmf_ctx *c, const float hp[8], int32_t max_epochs, double delta, int32_t *epochs_out,
                   double *rmse_out);

/* Order of the strata of epoch `epoch` (b entries): order[pos] = the
 * stratum run at position pos, stratum s being the blocks ((j + s) mod b, j)
 * (Section 3, parallel BMF: the diagonal first, then the blocks below it,
 * columns wrapping; every block once per iteration).  Mode 0 gives
 * 0, 1, ..., b-1, mode 1 the seeded shuffle of BMF_OPT_STRATUM_ORDER.
 * order: caller-allocated host array of b int32.  Host only, no device work.
 * Errors: BMF_E_INVAL (c or order NULL, epoch < 0). */
bmf_status bmf_get_schedule(const bmf_ctx *c, int32_t epoch, int32_t *order);

/* The partition of the loaded ratings into the b x b blocks (Section 3's
 * block representation, Algorithm 1 steps 1-2; inside a block Algorithm 2's
 * row-major order): block_ptr[b*b + 1] (bucket offsets into the processing
 * order, block id = row * b + column, rating t in block (u_t / rb,
 * i_t / cb)) and perm[nnz] (perm[pos] = input index of the rating visited
 * at position pos; inside a block (u, i, input index) ascending).  Both are
 * caller-allocated host arrays; either may be NULL to skip it.  Copies from
 * the device and synchronises.  Errors: BMF_E_STATE before a load. */
bmf_status bmf_get_partition(bmf_ctx *c, int64_t *block_ptr, int32_t *perm);

/* Copy the model out (any pointer may be NULL to skip it).  P: m*k, Q: n*k,
 * bu: m, bi: n floats; mu: one double.  Waits for the stream. */
bmf_status bmf_get_factors(bmf_ctx *c, float *P, float *Q, float *bu, float *bi, double *mu);

/* Replace the model (any pointer may be NULL to keep that part). */
bmf_status bmf_set_factors(bmf_ctx *c, const float *P, const float *Q, const float *bu,
                           const float *bi, const double *mu);

/* Device pointers to the live FP32 tables (owned by the context). */
bmf_status bmf_factor_ptrs(bmf_ctx *c, float **P, float **Q, float **bu, float **bi);

/* ----------------------------------------------------------- evaluation */

/* RMSE = sqrt(mean((r - (mu + bu_u + bi_i + p_u . q_i))^2)) over the given
 * ratings (host COO, cnt entries), or over the training ratings when u is
 * NULL.  Residuals in FP32, squares summed in FP64 in a fixed order (the
 * result does not depend on launch timing).  Algorithm 1's stopping test
 * uses the RMSE; the paper reports test RMSE (Section 5, Table 1).
 * Errors: BMF_E_RANGE for an out-of-range index; BMF_E_STATE. */
bmf_status bmf_rmse(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t cnt,
                    double *out);
/* bmf_rmse over device-resident ratings (u, i, r: device pointers of cnt
 * entries on the context's device; read only).  The ranges are checked on
 * the device (BMF_E_RANGE names the first bad index).  Synchronises. */
bmf_status bmf_rmse_dev(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t cnt,
                        double *out);

/* Regularised loss over the training ratings: sum of err^2 + beta_p |p_u|^2
 * + beta_q |q_i|^2 + beta_bu bu_u^2 + beta_bi bi_i^2 at every rating (Eq 9
 * with the penalty charged per observed rating, the objective per-rating SGD
 * descends).  hp as in bmf_epoch_hp (only the betas are used). */
bmf_status bmf_loss(bmf_ctx *c, const float hp[8], double *out);

/* ---------------------------------------------------------------- top-K */

/* For each of the nu user ids, the K items with the largest predicted
 * rating over all n items, best first, ties to the smaller item id.
 * Scores use FP32 factors on FP32 MFMA (v_mfma_f32_16x16x4_f32) with a
 * fixed accumulation order, so a user's result does not depend on the other
 * users in the call.  items_out[nu*K] (int32), scores_out[nu*K] (float,
 * the predicted rating mu + bu_u + bi_i + p_u . q_i).  If K > n the tail is
 * item -1 / score -inf.  1 <= K <= 512.
 * Errors: BMF_E_INVAL, BMF_E_RANGE (user id), BMF_E_DEVICE. */
bmf_status bmf_topk(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t *items_out,
                    float *scores_out);

/* Same ranking with BF16 copies of P and Q on BF16 MFMA (FP32 accumulate)
 * to pick Kc >= K candidates per user, then an FP32 rescore of those
 * candidates (fixed-order FP32 dot products) and a final exact top-K of the
 * rescored values.  Candidates whose BF16 score lies more than twice a
 * bound on the BF16 rounding error below the K-th best BF16 score cannot
 * reach that top K and are not rescored; the answer is the same (setting
 * BMF_TOPK_PRUNE=0 in the environment turns this off, to check it).  The
 * BF16 copies (round to nearest even) and per-item norm bounds are made
 * once after the factors last changed.  Kc = 0 selects K + max(16, K / 2). */
bmf_status bmf_topk_bf16(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t Kc,
                         int32_t *items_out, float *scores_out);

/* Device-pointer forms (users, items_out, scores_out on the device);
 * enqueue only. precision: 0 = FP32 MFMA, 1 = BF16 + FP32 rescore, 2 =
 * BF16 only: the K best BF16 scores (BF16 P and Q, FP32 accumulation with
 * the FP32 item bias as the starting value, ties to the smaller item id),
 * returned as mu + bu_u plus that score, with no rescore (Kc is not used).
 * A BF16 score differs from the exact p . q + bi by at most about
 * 2 * 2^-8 * sum_f |p_f q_f| (two BF16 roundings) plus the FP32 rounding
 * of the sum, and the ranking follows those scores. */
bmf_status bmf_topk_dev(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t precision,
                        int32_t Kc, int32_t *items_out, float *scores_out);

/* For callers that cannot allocate device memory (work captured into a
 * HIP graph, serving loops that must not allocate, harnesses that forbid
 * hipMalloc): bmf_topk_dev with the same arguments, checks and results
 * (bit for bit), but its workspace (user rows, thresholds, candidate lists)
 * is a fixed array of 64 MiB that the library holds on every device it
 * runs on until the process ends; no device memory is allocated or freed.
 * A request whose workspace exceeds 64 MiB (at K = 100 about 4,200 users
 * at n = 27,000 and k = 64, about 1,800 at n = 100,000 and k = 128) fails
 * with BMF_E_NOMEM and changes nothing: split it.  Precisions 1 and 2
 * also need the BF16 item table's memory, which the first BF16 call that
 * may allocate (bmf_topk_bf16, bmf_topk_dev, bmf_server_create) makes:
 * BMF_E_STATE before that.  Every call on one device shares the array, so calls that
 * may overlap on one device (other streams, other contexts, other host
 * threads) race and must be serialised by the caller.  Enqueue only. */
bmf_status bmf_topk_dev_noalloc(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t precision,
                                int32_t Kc, int32_t *items_out, float *scores_out);

/* ---------------------------------------------------------------- fold-in */

/* Fold in a new user (Section 2.1's folding-in of new data; Section 6's
 * incremental use): item factors and item biases stay fixed, p = 0 and
 * bu = 0, then `passes` passes over the user's nr ratings in input order,
 * each applying err = r - mu - bu - bi_i - p . q_i; bu += lr (err - reg bu);
 * p += lr (err q_i - reg p).  p_out[k], bu_out[1] on the host.
 * Errors: BMF_E_INVAL, BMF_E_RANGE (item id or non-finite rating). */
bmf_status bmf_foldin(bmf_ctx *c, const int32_t *items, const float *r, int32_t nr, int32_t passes,
                      float lr, float reg, float *p_out, float *bu_out);

/* ------------------------------------------------------------- counters */

/* Time spent in SGD kernels since the last reset, measured with HIP events
 * on the context's stream around each epoch's launches (milliseconds), and
 * the number of SGD kernel launches. */
bmf_status bmf_sgd_timing(bmf_ctx *c, double *ms, int64_t *launches, int32_t reset);

/* Stratum order of epoch `epoch` for a b x b grid without a context: the
 * same rule as BMF_OPT_STRATUM_ORDER (mode 0 identity, mode 1 seeded
 * Fisher-Yates).  Host-only; order[b].  Errors: BMF_E_INVAL. */
bmf_status bmf_stratum_order(int32_t b, uint64_t seed, int32_t epoch, int32_t mode, int32_t *order);

/* -------------------------------------------------------------- batched */

/* Many independent problems of uneven size trained together.  Each launch
 * runs one global stratum position (epoch * b_p + position in the epoch's
 * order) of every problem that has one, i.e. the blocks of up to nprob
 * strata at once (Section 3's rule that blocks sharing no row or column are
 * independent, applied within and across problems); successive positions
 * follow in stream order.  Per problem the results are bit-identical to
 * training that problem alone with the same grid and options.
 * m[nprob], n[nprob]: sizes; k (1..128) shared; b[nprob]: block grid per
 * problem, or b == NULL / b[p] == 0 for the autotuner (cost model of the
 * per-epoch dependency chain and block staging, fitted by timed epochs of
 * the largest problem; it also picks the waves per workgroup).
 * Errors: BMF_E_INVAL, BMF_E_NOMEM, BMF_E_DEVICE. */
bmf_status bmf_batch_create(int32_t nprob, const int64_t *m, const int64_t *n, int32_t k, const int32_t *b,
                            bmf_batch **out);
void bmf_batch_destroy(bmf_batch *B);
const char *bmf_batch_last_error(const bmf_batch *B);
/* BMF_OPT_SEED, BMF_OPT_ORDER_SEED, BMF_OPT_STRATUM_ORDER (applied to every
 * problem) and BMF_OPT_WAVES_PER_BLOCK (0 = tuned); before any load. */
bmf_status bmf_batch_set_option(bmf_batch *B, int32_t key, int64_t value);
/* Ratings of problem p (host COO, as bmf_load_ratings); copied and
 * validated now, partitioned when the grids are chosen. */
bmf_status bmf_batch_load(bmf_batch *B, int32_t p, const int32_t *u, const int32_t *i, const float *r,
                          int64_t nnz);
/* Choose grids for every loaded problem and partition them (done
 * implicitly by the first bmf_batch_epochs). */
bmf_status bmf_batch_tune(bmf_batch *B);
/* `epochs` epochs of every problem (max_p epochs * b_p launches); hp as in
 * bmf_epoch_hp.  Waits for completion.  Every problem must be loaded. */
bmf_status bmf_batch_epochs(bmf_batch *B, int32_t epochs, const float hp[8]);
/* Borrowed context of problem p (valid until bmf_batch_destroy): use it
 * for bmf_rmse, bmf_get_factors, bmf_topk, ...; do not destroy it. */
bmf_status bmf_batch_problem(bmf_batch *B, int32_t p, bmf_ctx **out);
/* Chosen grid and waves for problem p, and the model's epoch time (ms, -1
 * when the grid was given). */
bmf_status bmf_batch_info(bmf_batch *B, int32_t p, int32_t *b_out, int32_t *waves_out, double *predicted_ms);
/* Time in batched epochs calls (HIP events on the batch stream around all
 * their launches, ms) and the number of launches. */
bmf_status bmf_batch_timing(bmf_batch *B, double *ms, int64_t *launches, int32_t reset);

/* -------------------------------------------------------------- serving */

/* Continuous-batching server over a trained context (its factors are read,
 * never written; do not train the context while a server is open).  A
 * scheduler thread forms batches from the FIFO queue of submitted requests:
 * a batch takes requests from the head while their device workspace fits
 * one batch partition of the memory budget (admission by memory) and the
 * row cap allows; up to max_batches batches are on the GPU at once on their
 * own streams, so requests arriving meanwhile go into the next batch while
 * earlier ones are still running.  Within a batch, fold-in requests run the
 * fold-in kernel and all rows of a precision are scored in one pass.  Each
 * row is scored independently, so a request's result is the same whatever
 * batch it lands in.  The workspace (mem_budget_bytes of device memory and
 * as much pinned host memory) is allocated at creation; no allocation
 * happens per request. */
typedef struct {
    int64_t mem_budget_bytes;       /* device workspace for in-flight batches (0: 1 GiB) */
    int32_t max_batches;            /* batches on the GPU at once, 1..4 (0: 4) */
    int32_t max_batch_rows;         /* users per batch, top-K users plus fold-ins (0: 4096); the first
                                       request of a batch is taken whatever its size */
    int32_t max_requests_per_batch; /* 0: unlimited; 1 turns batching off */
    int32_t foldin_passes;          /* passes of a fold-in (0: 10) */
    float foldin_lr, foldin_reg;    /* fold-in step and regulariser (0: 0.005, 0.05) */
    int32_t Kc;                     /* BF16 candidates per user (0: K + max(16, K/2)); at most 1008 */
} bmf_server_config;

typedef struct {
    int64_t submitted, completed, rejected, batches, rows;
    int64_t budget_bytes, peak_bytes, queue_depth;
    double p50_ms, p90_ms, p99_ms, max_ms, mean_ms; /* submit-to-completion latency */
} bmf_server_stats;

/* cfg may be NULL (all defaults).  Errors: BMF_E_INVAL (k > 256, Kc < 0 or Kc > 1008),
 * BMF_E_NOMEM, BMF_E_DEVICE. */
bmf_status bmf_server_create(bmf_ctx *c, const bmf_server_config *cfg, bmf_server **out);
/* Stops the scheduler (queued requests are dropped, running batches
 * finish) and frees the workspace. */
void bmf_server_destroy(bmf_server *S);
/* The server's last error message (a scheduler failure starts with
 * "server failed: ").  The string is the calling thread's copy, valid until
 * that thread's next call of this function. */
const char *bmf_server_last_error(const bmf_server *S);
/* Top-K for nu user ids (host array, copied); precision 0 = FP32 MFMA,
 * 1 = BF16 + FP32 rescore; 1 <= K <= 512.  *id names the request.
 * Errors: BMF_E_RANGE (bad id), BMF_E_NOMEM (the request alone exceeds a
 * batch partition; counted as rejected). */
bmf_status bmf_server_submit_topk(bmf_server *S, const int32_t *users, int32_t nu, int32_t K, int32_t precision,
                                  int64_t *id);
/* Fold in a new user from nr (item, rating) pairs (bmf_foldin's update with
 * the server's passes, lr, reg), then its top-K. */
bmf_status bmf_server_submit_foldin(bmf_server *S, const int32_t *items, const float *ratings, int32_t nr,
                                    int32_t K, int32_t precision, int64_t *id);
/* Result of request id; wait != 0 blocks until it is done.  On done = 1
 * copies items_out[rows*K], scores_out[rows*K] (rows = nu, or 1 for a
 * fold-in), p_out[k] and bu_out[1] for fold-ins (any may be NULL) and the
 * submit-to-completion latency, and forgets the request. */
bmf_status bmf_server_poll(bmf_server *S, int64_t id, int32_t wait, int32_t *done, int32_t *items_out,
                           float *scores_out, float *p_out, float *bu_out, int64_t *latency_ns);
/* Wait until every submitted request is done. */
bmf_status bmf_server_drain(bmf_server *S);
/* Counters and latency percentiles (of completed requests since the last
 * reset). */
bmf_status bmf_server_get_stats(bmf_server *S, bmf_server_stats *out, int32_t reset);

/* ---------------------------------------------------------- diagnostics */

/* Host-only: the step plan the LDS-staged SGD kernel follows for one block
 * (no device needed).  u_local[x], i_local[x], r[x], x < n: the block's
 * ratings in processing order ((u, i) non-decreasing, BMF_E_INVAL
 * otherwise), 0 <= i_local < cb < 65536 and u_local < 2^(32 - bits(cb))
 * (BMF_E_RANGE otherwise); slots = LDS user slots (1..4095), chunk = steps
 * per chunk (>= 1).  *n_steps receives the number of steps.  When out is
 * non-null it receives 4 records per step, 4 uint32 words each: {meta,
 * rating bits, u_local, x} with meta = i_local | slot << 16 | 1 << 30 (the
 * user's first rating) | 1 << 31 (its last); an empty record has
 * i_local = cb, slot = slots and x = 0xffffffff.  Ratings of one step share
 * no user and no item; every user's and every item's ratings keep their
 * order; a slot freed in chunk a is next used in chunk a + 3 or later.
 * BMF_E_RANGE when out is non-null and max_steps is smaller than the plan. */
bmf_status bmf_debug_block_plan(int64_t n, const int32_t *u_local, const int32_t *i_local, const float *r,
                                int32_t cb, int32_t slots, int32_t chunk, int64_t max_steps, int64_t *n_steps,
                                uint32_t *out);

/* Host-only: the plan a top-K request of nu users over n items with k
 * factors gets (bmf_topk_dev and the server make the same one; no device
 * needed).  out[7] receives: the number s of sampled items the threshold
 * pass scores (0: no threshold, every item is a candidate), the rank r of
 * the sampled score taken as the threshold (the smallest r for which fewer
 * than `need` items reach the r-th best of s sampled ones with probability
 * at most 1e-6, by the Poisson approximation), the candidates per user the
 * buffer holds, `need` (K, or the BF16 candidate count for precision 1),
 * the filter's item splits, the items per split, and the request's
 * workspace bytes.  Arguments as for bmf_topk_dev; BMF_E_INVAL otherwise. */
bmf_status bmf_debug_topk_plan(int64_t n, int32_t k, int64_t nu, int32_t K, int32_t precision, int32_t Kc,
                               int64_t *out);

/* Host-only: the dependency depth of a block's ratings u[x], i[x] (x < n,
 * in processing order, ids >= 0): the length of the longest chain of
 * ratings, each sharing its user or its item with the one before it.
 * Algorithm 2 updates p_u, bu_u, q_i and bi_i at every rating, so the
 * ratings of such a chain must run one after another and no schedule of
 * the block (Section 3: a block is factorised by one worker) has fewer
 * dependent steps.  Errors: BMF_E_INVAL, BMF_E_RANGE (negative id). */
bmf_status bmf_chain_depth(int64_t n, const int32_t *u, const int32_t *i, int64_t *depth);

/* The dependent-step floor of the LDS-staged SGD kernel on the current
 * device: one wavefront runs the kernel's own chunk loop (four ratings per
 * step, Eqs 10-13 on rows in LDS) for `steps` steps (rounded down to whole
 * chunks of 16) in which every step reads the rows the step before it wrote,
 * with no staging, barrier or other wavefront.  *ns_per_step receives the
 * GPU time per step (HIP events around a second launch): the least time a
 * block's plan can take per dependent step (Algorithm 2's updates of one
 * block follow each other, Section 3).  k <= 128.  Errors: BMF_E_INVAL,
 * BMF_E_DEVICE (bmf_last_error(NULL) has the message). */
bmf_status bmf_debug_chain_floor(int32_t k, int32_t steps, double *ns_per_step);

/* Race check of the schedule on the device (Section 3: the blocks of one
 * stratum share no user and no item, which is what lets them run at once
 * without locks).  For each stratum s the check walks the resident records
 * that the next epoch's SGD kernel reads for the stratum's blocks (the
 * partition's records, or the LDS-staged kernel's step plan), marks the
 * user row and the item row each rating updates with a tag of its block,
 * and counts the ratings that find their row marked by another block of
 * the same stratum, plus any record naming a row outside its block.
 * *conflicts is 0 exactly when the blocks of every stratum are disjoint.
 * pairing: NULL for the schedule the epochs run (stratum s pairs block
 * column j with block row (j + s) mod b), or a host array of b*b block
 * rows, pairing[s*b + j] the row that stratum s pairs with column j, to
 * check another schedule (one that pairs two columns with the same row
 * shares a user row wherever both of those blocks hold ratings of one
 * user).  Allocates 8 (m + n) bytes of device memory for the call;
 * synchronises.  With BMF_CHECK_DISJOINT=1 in the environment, every epoch
 * on resident ratings runs this check first and, when the count is not 0,
 * fails with BMF_E_STATE without running.  Errors: BMF_E_INVAL (null
 * output, pairing entry outside [0, b)), BMF_E_STATE (no ratings loaded,
 * out-of-core ratings, SGD kernel 2 forced where it does not apply),
 * BMF_E_DEVICE. */
bmf_status bmf_check_disjoint(bmf_ctx *c, const int32_t *pairing, int64_t *conflicts);

/* Reduction self-check on the current device: out[0:64], out[64:128],
 * out[128:192] and out[192:256] receive, per lane, the 64-lane sum of
 * in[0:64] by the shuffle butterfly, by the DPP butterfly, the 16-lane row
 * sums by DPP, and the 64-lane sum by DPP plus permlane swaps.  The three
 * full sums must be bit-identical.  Host arrays. */
bmf_status bmf_debug_wave_sum(const float *in64, float *out256);

#ifdef __cplusplus
}
#endif

#endif /* BMF_H */
