/*
 * oracle.c -- plain, slow FP64 reference of block-based biased-SVD SGD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP library: every
 * routine here is written out from the paper's definitions.
 *
 * Paper: Bhavana, Kumar, Padmanabhan, "Block based Singular Value
 * Decomposition approach to matrix factorization for recommender systems"
 * (arXiv 1907.07410).
 *
 * Notation: m users (rows of X), n items (columns), k latent factors,
 * b x b block grid, P (m x k) user factors, Q (n x k) item factors, bu, bi
 * biases, mu global mean.  All state is FP64, row-major.
 *
 * Readings of the paper used here (where it is garbled or silent):
 *  - prediction mu + bu_u + bi_i + p_u . q_i (Eq 3 plus a global mean; the
 *    mean can be switched off to get Eq 3 literally);
 *  - Eqs 10-13 read as  x += alpha * (err * other - beta * x): the gradient
 *    of the regularised objective (Eq 9) with the factor 2 absorbed;
 *  - Eq 11's q_u is q_i; the bias regularisers use the bias being updated
 *    (Eqs 12-13), not the crossed ones of Algorithm 2;
 *  - all four updates use the residual and the values from before the
 *    update (simultaneous form).  Two other forms are kept as a switch:
 *    the Gauss-Seidel factor order of Algorithm 2 (item factors updated
 *    with the new user factor), and Algorithm 2 as printed, which also
 *    penalises the user bias with the item bias and the item bias with
 *    the user bias it has just updated;
 *  - block extents rb = ceil(m/b), cb = ceil(n/b) (Section 5's 755 x 486
 *    example for 6040 users and b = 8);
 *  - stratum s = {((j + s) mod b, j)} (Section 3, parallel BMF: diagonal
 *    first, then the block below in each column, wrapping);
 *  - inside a block ratings are visited row-major, (u asc, i asc), and
 *    duplicates in input order (Algorithm 2's row/column loops).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG
 * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), used counter-style: draw j of the stream with
 * seed s is mix(s + (j + 1) * gamma).  The method draws random numbers in
 * two places: the initial factors (Algorithm 1, "random values") and the
 * optional seeded stratum order.                                        */
static const uint64_t GOLDEN = 0x9E3779B97F4A7C15ULL;

static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t j)
{
    return sm_mix(seed + (j + 1) * GOLDEN);
}

/* Initial factor entry for tensor tag T (1 user factors, 2 item factors):
 * x = draw (row*k + f) of stream seed ^ (T << 56);
 * value = 0.125 * (2 * (x >> 40) * 2^-24 - 1), a value in [-0.125, 0.125)
 * that is exact in FP32 and FP64.                                       */
double orc_init_value(uint64_t seed, int tag, int64_t row, int k, int f)
{
    uint64_t x = orc_splitmix64(seed ^ ((uint64_t)tag << 56), (uint64_t)row * (uint64_t)k + (uint64_t)f);
    double u01 = (double)(x >> 40) * (1.0 / 16777216.0);
    return 0.125 * (2.0 * u01 - 1.0);
}

void orc_init_factors(int64_t m, int64_t n, int k, uint64_t seed, double *P, double *Q,
                      double *bu, double *bi)
{
    for (int64_t u = 0; u < m; ++u) {
        for (int f = 0; f < k; ++f) P[u * k + f] = orc_init_value(seed, 1, u, k, f);
        bu[u] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int f = 0; f < k; ++f) Q[i * k + f] = orc_init_value(seed, 2, i, k, f);
        bi[i] = 0.0;
    }
}

/* Global mean of the training ratings, summed in input order. */
double orc_mean(const float *r, int64_t nnz)
{
    double s = 0.0;
    for (int64_t t = 0; t < nnz; ++t) s += (double)r[t];
    return nnz > 0 ? s / (double)nnz : 0.0;
}

/* ------------------------------------------------------------ partition
 * Block (br, bc) of rating t is (u / rb, i / cb); block id br * b + bc.
 * block_ptr[b*b + 1] holds bucket offsets; perm[pos] is the input index of
 * the rating visited at processing position pos.  Inside a block the order
 * is (u asc, i asc, input index asc).                                    */
typedef struct {
    const int32_t *u, *i;
} sort_ctx;
static sort_ctx g_sort;

static int cmp_rating(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_sort.u[x] != g_sort.u[y]) return g_sort.u[x] < g_sort.u[y] ? -1 : 1;
    if (g_sort.i[x] != g_sort.i[y]) return g_sort.i[x] < g_sort.i[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int orc_partition(int64_t m, int64_t n, int b, const int32_t *u, const int32_t *i, int64_t nnz,
                  int64_t *block_ptr, int32_t *perm)
{
    if (b < 1 || m < 1 || n < 1) return -1;
    int64_t rb = (m + b - 1) / b, cb = (n + b - 1) / b;
    int64_t nb = (int64_t)b * b;
    int64_t *cnt = calloc((size_t)nb + 1, sizeof(int64_t));
    if (!cnt) return -4;
    for (int64_t t = 0; t < nnz; ++t) {
        int64_t blk = (u[t] / rb) * b + (i[t] / cb);
        cnt[blk + 1]++;
    }
    for (int64_t q = 0; q < nb; ++q) cnt[q + 1] += cnt[q];
    memcpy(block_ptr, cnt, (size_t)(nb + 1) * sizeof(int64_t));
    /* place input indices into their buckets in input order */
    for (int64_t t = 0; t < nnz; ++t) {
        int64_t blk = (u[t] / rb) * b + (i[t] / cb);
        perm[cnt[blk]++] = (int32_t)t;
    }
    free(cnt);
    g_sort.u = u;
    g_sort.i = i;
    for (int64_t q = 0; q < nb; ++q) {
        int64_t s = block_ptr[q], e = block_ptr[q + 1];
        if (e - s > 1) qsort(perm + s, (size_t)(e - s), sizeof(int32_t), cmp_rating);
    }
    return 0;
}

/* ------------------------------------------------------------- schedule
 * Order of strata in epoch e.  mode 0: 0, 1, ..., b-1 (the paper's
 * diagonal-first order).  mode 1: Fisher-Yates shuffle of 0..b-1 driven by
 * the SplitMix64 stream seed ^ (3 << 56) ^ (e << 24): for t = b-1 down to
 * 1, j = draw(b-1-t) mod (t+1), swap entries t and j.                    */
void orc_schedule(int b, uint64_t seed, int epoch, int mode, int32_t *order)
{
    for (int s = 0; s < b; ++s) order[s] = s;
    if (mode == 0) return;
    uint64_t stream = seed ^ (3ULL << 56) ^ ((uint64_t)(uint32_t)epoch << 24);
    for (int t = b - 1; t >= 1; --t) {
        uint64_t x = orc_splitmix64(stream, (uint64_t)(b - 1 - t));
        int j = (int)(x % (uint64_t)(t + 1));
        int32_t tmp = order[t];
        order[t] = order[j];
        order[j] = tmp;
    }
}

/* ---------------------------------------------------------------- update
 * One observed rating (Eqs 10-13).  hp[8] = {alpha_p, beta_p, alpha_q,
 * beta_q, alpha_bu, beta_bu, alpha_bi, beta_bi} (user-latent, item-latent,
 * user-bias, item-bias).
 * form 0: Eqs 10-13 with every right-hand side taken before the update;
 * form 1: the same biases, item factors from the updated user factors
 *         (Algorithm 2's statement order for U and V);
 * form 2: Algorithm 2 as printed: the user bias is penalised by the item
 *         bias, the item bias by the user bias just updated, and the item
 *         factors use the updated user factors.                          */
enum { FORM_SIMULTANEOUS = 0, FORM_GAUSS_SEIDEL = 1, FORM_ALG2_LITERAL = 2 };

typedef struct {
    int64_t m, n;
    int k;
    double *P, *Q, *bu, *bi;
    double mu;
    double hp[8];
    int form;
} orc_state;

static void update_one(orc_state *S, int64_t u, int64_t i, double r)
{
    const int k = S->k;
    double *p = S->P + u * k, *q = S->Q + i * k;
    double dot = 0.0;
    for (int f = 0; f < k; ++f) dot += p[f] * q[f];
    double err = r - S->mu - S->bu[u] - S->bi[i] - dot;
    double bu0 = S->bu[u], bi0 = S->bi[i];
    if (S->form == FORM_ALG2_LITERAL) {
        double bun = bu0 + S->hp[4] * (err - S->hp[5] * bi0);
        S->bu[u] = bun;
        S->bi[i] = bi0 + S->hp[6] * (err - S->hp[7] * bun);
    } else {
        S->bu[u] = bu0 + S->hp[4] * (err - S->hp[5] * bu0);
        S->bi[i] = bi0 + S->hp[6] * (err - S->hp[7] * bi0);
    }
    for (int f = 0; f < k; ++f) {
        double pf = p[f], qf = q[f];
        double pn = pf + S->hp[0] * (err * qf - S->hp[1] * pf);
        double pq = S->form == FORM_SIMULTANEOUS ? pf : pn;
        p[f] = pn;
        q[f] = qf + S->hp[2] * (err * pq - S->hp[3] * qf);
    }
}

typedef struct {
    orc_state *S;
    const int32_t *u, *i;
    const float *r;
    const int64_t *block_ptr;
    const int32_t *perm;
    int b, stratum, j0, j1;
} block_job;

static void run_block(orc_state *S, const int32_t *u, const int32_t *i, const float *r,
                      const int64_t *block_ptr, const int32_t *perm, int64_t blk)
{
    for (int64_t pos = block_ptr[blk]; pos < block_ptr[blk + 1]; ++pos) {
        int32_t t = perm[pos];
        update_one(S, u[t], i[t], (double)r[t]);
    }
}

static void *stratum_worker(void *arg)
{
    block_job *J = (block_job *)arg;
    for (int j = J->j0; j < J->j1; ++j) {
        int64_t br = (j + J->stratum) % J->b, bc = j;
        run_block(J->S, J->u, J->i, J->r, J->block_ptr, J->perm, br * J->b + bc);
    }
    return NULL;
}

/* One epoch (Algorithm 1's loop body): every stratum in the epoch's order,
 * every block of the stratum, every rating of the block.  The blocks of a
 * stratum share no user and no item, so with threads > 1 they are spread
 * over threads with a join after each stratum (the CPU block variant of
 * Section 5); results are identical for every thread count.             */
int orc_epoch(int64_t m, int64_t n, int k, int b, double *P, double *Q, double *bu, double *bi,
              double mu, const double *hp, int form, const int32_t *u, const int32_t *i,
              const float *r, const int64_t *block_ptr, const int32_t *perm, const int32_t *order,
              int threads)
{
    if (form < FORM_SIMULTANEOUS || form > FORM_ALG2_LITERAL) return -1;
    orc_state S = {m, n, k, P, Q, bu, bi, mu, {0}, form};
    memcpy(S.hp, hp, sizeof(S.hp));
    if (threads < 1) threads = 1;
    if (threads > b) threads = b;
    pthread_t tid[256];
    block_job jobs[256];
    if (threads > 256) threads = 256;
    for (int pos = 0; pos < b; ++pos) {
        int s = order[pos];
        if (threads == 1) {
            for (int j = 0; j < b; ++j) {
                int64_t br = (j + s) % b;
                run_block(&S, u, i, r, block_ptr, perm, br * b + j);
            }
            continue;
        }
        for (int w = 0; w < threads; ++w) {
            jobs[w] = (block_job){&S, u, i, r, block_ptr, perm, b, s, (int)((int64_t)b * w / threads),
                                  (int)((int64_t)b * (w + 1) / threads)};
            if (pthread_create(&tid[w], NULL, stratum_worker, &jobs[w]) != 0) return -5;
        }
        for (int w = 0; w < threads; ++w) pthread_join(tid[w], NULL);
    }
    return 0;
}

/* ------------------------------------------------------------ evaluation
 * RMSE = sqrt(mean((r - xhat)^2)) over the given ratings, unclipped.
 * Loss = sum over ratings of err^2 + beta_p |p_u|^2 + beta_q |q_i|^2
 *        + beta_bu bu_u^2 + beta_bi bi_i^2
 * (Eq 9 with the penalty taken at every observed rating, which is the
 * objective that per-rating SGD descends).                               */
static double predict(int k, const double *P, const double *Q, const double *bu, const double *bi,
                      double mu, int64_t u, int64_t i)
{
    double dot = 0.0;
    for (int f = 0; f < k; ++f) dot += P[u * k + f] * Q[i * k + f];
    return mu + bu[u] + bi[i] + dot;
}

double orc_rmse(int k, const double *P, const double *Q, const double *bu, const double *bi, double mu,
                const int32_t *u, const int32_t *i, const float *r, int64_t cnt)
{
    double s = 0.0;
    for (int64_t t = 0; t < cnt; ++t) {
        double e = (double)r[t] - predict(k, P, Q, bu, bi, mu, u[t], i[t]);
        s += e * e;
    }
    return cnt > 0 ? sqrt(s / (double)cnt) : 0.0;
}

double orc_loss(int k, const double *P, const double *Q, const double *bu, const double *bi, double mu,
                const double *hp, const int32_t *u, const int32_t *i, const float *r, int64_t cnt)
{
    double s = 0.0;
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t uu = u[t], ii = i[t];
        double e = (double)r[t] - predict(k, P, Q, bu, bi, mu, uu, ii);
        double pp = 0.0, qq = 0.0;
        for (int f = 0; f < k; ++f) {
            pp += P[uu * k + f] * P[uu * k + f];
            qq += Q[ii * k + f] * Q[ii * k + f];
        }
        s += e * e + hp[1] * pp + hp[3] * qq + hp[5] * bu[uu] * bu[uu] + hp[7] * bi[ii] * bi[ii];
    }
    return s;
}

/* ----------------------------------------------------------------- top-K
 * For each requested user, the K items with the largest predicted rating
 * mu + bu_u + bi_i + p_u . q_i over all n items, in descending order of
 * score, ties broken by the smaller item id.  Full sort, FP64.           */
typedef struct {
    double s;
    int32_t item;
} scored;

static int cmp_scored(const void *a, const void *b)
{
    const scored *x = a, *y = b;
    if (x->s != y->s) return x->s > y->s ? -1 : 1;
    return x->item < y->item ? -1 : (x->item > y->item ? 1 : 0);
}

int orc_topk(int64_t n, int k, const double *P, const double *Q, const double *bu, const double *bi,
             double mu, const int32_t *users, int64_t nu, int K, int32_t *items_out,
             double *scores_out)
{
    scored *buf = malloc((size_t)n * sizeof(scored));
    if (!buf) return -4;
    for (int64_t q = 0; q < nu; ++q) {
        int64_t u = users[q];
        for (int64_t i = 0; i < n; ++i) {
            buf[i].s = predict(k, P, Q, bu, bi, mu, u, i);
            buf[i].item = (int32_t)i;
        }
        qsort(buf, (size_t)n, sizeof(scored), cmp_scored);
        for (int j = 0; j < K; ++j) {
            items_out[q * K + j] = j < n ? buf[j].item : -1;
            scores_out[q * K + j] = j < n ? buf[j].s : -INFINITY;
        }
    }
    free(buf);
    return 0;
}

/* Same ranking for a single explicit user vector (p, bu), e.g. a folded-in
 * user. */
int orc_topk_vec(int64_t n, int k, const double *p, double bu_u, const double *Q, const double *bi,
                 double mu, int K, int32_t *items_out, double *scores_out)
{
    scored *buf = malloc((size_t)n * sizeof(scored));
    if (!buf) return -4;
    for (int64_t i = 0; i < n; ++i) {
        double dot = 0.0;
        for (int f = 0; f < k; ++f) dot += p[f] * Q[i * k + f];
        buf[i].s = mu + bu_u + bi[i] + dot;
        buf[i].item = (int32_t)i;
    }
    qsort(buf, (size_t)n, sizeof(scored), cmp_scored);
    for (int j = 0; j < K; ++j) {
        items_out[j] = j < n ? buf[j].item : -1;
        scores_out[j] = j < n ? buf[j].s : -INFINITY;
    }
    free(buf);
    return 0;
}

/* --------------------------------------------------------------- fold-in
 * Folding-in a new user (Section 2.1's folding-in, Section 6's incremental
 * use): item factors and item biases stay fixed; p and bu start at zero
 * and take `passes` passes of the per-rating updates (Eqs 10 and 12) over
 * the user's ratings in input order.                                     */
void orc_foldin(int k, const double *Q, const double *bi, double mu, const int32_t *items,
                const float *r, int64_t cnt, int passes, const double *hp, double *p_out,
                double *bu_out)
{
    double bu = 0.0;
    for (int f = 0; f < k; ++f) p_out[f] = 0.0;
    for (int pass = 0; pass < passes; ++pass) {
        for (int64_t t = 0; t < cnt; ++t) {
            const double *q = Q + (int64_t)items[t] * k;
            double dot = 0.0;
            for (int f = 0; f < k; ++f) dot += p_out[f] * q[f];
            double err = (double)r[t] - mu - bu - bi[items[t]] - dot;
            bu = bu + hp[4] * (err - hp[5] * bu);
            for (int f = 0; f < k; ++f) p_out[f] = p_out[f] + hp[0] * (err * q[f] - hp[1] * p_out[f]);
        }
    }
    *bu_out = bu;
}

/* ------------------------------------------------------------------ BF16
 * Round-to-nearest-even conversion of an FP32 value to bfloat16 (the top
 * 16 bits of the FP32 pattern after rounding), returned as the FP32 value
 * it represents.  NaN stays NaN.                                         */
float orc_bf16_round(float x)
{
    uint32_t bits;
    memcpy(&bits, &x, 4);
    if ((bits & 0x7f800000u) == 0x7f800000u && (bits & 0x007fffffu)) {
        bits |= 0x00400000u;
    } else {
        uint32_t lsb = (bits >> 16) & 1u;
        bits += 0x7fffu + lsb;
    }
    bits &= 0xffff0000u;
    float y;
    memcpy(&y, &bits, 4);
    return y;
}

/* orc_bf16_round over an array: y[t] = orc_bf16_round(x[t]).            */
void orc_bf16_round_n(const float *x, float *y, int64_t count)
{
    for (int64_t t = 0; t < count; ++t) y[t] = orc_bf16_round(x[t]);
}
