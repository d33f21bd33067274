// Batched training: many independent factorisation problems of uneven size
// trained together (the block independence of Section 3 applied across
// problems: blocks of different problems never share data), with the block
// grid of every problem and the waves per workgroup chosen by an autotuner.
// One launch runs one global stratum position of every problem that has
// one, so a launch holds the blocks of up to sum_p b_p strata at once.
//
// Autotuner.  For problem p and grid b the epoch time is modelled as
//   T_p(b) = c_r * crit_p(b) + b * (c_s * cb * k + c_f)
// where crit_p(b) = sum over strata of the largest block's rating count
// (the dependent update chain when one workgroup runs each block), cb * k
// the item slice a block stages, and c_r, c_s, c_f per-device constants
// fitted from timed epochs of the largest problem at three grids (cached
// per device and k).  All problems share the GPU, so the batch time is at
// least the total work W = sum_p [nnz_p * c_r + b_p^2 * (c_s * cb * k +
// c_f)] divided by the number of resident workgroups; the tuner first takes
// each problem's fastest grid, then lowers grids that are faster than that
// bound (fewer, larger blocks cost less staging) as long as they stay under
// it.  The waves per workgroup (4 or 8: one wave runs the update chain, the
// others stage data) are picked by timing both on the largest problem.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>

#include "internal.h"

using namespace bmf;

namespace {
// A problem's ratings on the device, validated, kept until its grid is
// chosen and its context loaded.
struct Loaded {
    DevBuf u, i, r;
    int64_t nnz = 0;
};
}  // namespace

struct bmf_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int k = 0;
    std::vector<int64_t> m, n;
    std::vector<int32_t> b_req;
    std::vector<bmf_ctx *> probs;  // one context per problem (null until loaded)
    std::vector<double> predicted_ms;
    int waves = 0;  // 0 = not chosen yet
    uint64_t seed = 1001, order_seed = 2001;
    int order_mode = 0;
    double ms = 0.0;
    int64_t launches = 0;
    bool poisoned = false;
    std::string err;
    DevBuf d_probs, d_items;
    std::vector<std::unique_ptr<Loaded>> staged;  // per problem, until tuned
};

namespace {

struct Coef {
    double c_r = 150e-9, c_s = 2e-12, c_f = 5e-6;  // seconds; replaced by the fitted values
    bool fitted = false;
};
std::mutex g_coef_mu;
std::map<std::pair<int, int>, Coef> g_coef;  // (device, k) -> constants

int64_t critical_path(const std::vector<int64_t> &cnt, int b) {
    int64_t tot = 0;
    for (int s = 0; s < b; ++s) {
        int64_t mx = 0;
        for (int j = 0; j < b; ++j) mx = std::max(mx, cnt[(int64_t)((j + s) % b) * b + j]);
        tot += mx;
    }
    return tot;
}

struct Candidate {
    int b;
    int64_t crit;
    int64_t cb;
};

bool grid_ok(int64_t m, int64_t n, int k, int b, int device) {
    const int64_t rb = (m + b - 1) / b, cb = (n + b - 1) / b;
    int ub = 0, ib = 0;
    while ((1ll << ub) < rb) ++ub;
    while ((1ll << ib) < cb) ++ib;
    if (ub + ib > 32) return false;
    const int kp = plan_kp(k);
    return kp && cb + 1 <= (1 << 16) && plan_slots(kp, cb, PLAN_CH, sgd_max_lds(device)) >= PLAN_MIN_SLOTS;
}

double model_ms(const Coef &c, const Candidate &x, int k) {
    return 1e3 * (c.c_r * (double)x.crit + (double)x.b * (c.c_s * (double)x.cb * k + c.c_f));
}

double work_ms(const Coef &c, const Candidate &x, int k, int64_t nnz) {
    return 1e3 * (c.c_r * (double)nnz + (double)x.b * x.b * (c.c_s * (double)x.cb * k + c.c_f));
}

// Time one epoch (after one warm-up epoch) of a scratch context holding the
// given device ratings.
double time_epoch(int64_t m, int64_t n, int k, int b, int waves, const int32_t *du, const int32_t *di,
                  const float *dr, int64_t nnz, hipStream_t) {
    bmf_ctx *c = nullptr;
    if (bmf_create(m, n, k, b, &c) != BMF_OK) BMF_FAIL(BMF_E_DEVICE, "autotuner probe: create failed");
    std::unique_ptr<bmf_ctx, void (*)(bmf_ctx *)> guard(c, bmf_destroy);
    c->M.waves = waves;
    if (bmf_load_ratings_dev(c, du, di, dr, nnz) != BMF_OK) BMF_FAIL(BMF_E_DEVICE, "autotuner probe: " + c->err);
    bmf_epoch(c, 0.f, 0.f);  // lr = 0 keeps the scratch factors unchanged; timing is the same
    double ms = 0;
    int64_t l = 0;
    bmf_sgd_timing(c, &ms, &l, 1);
    if (bmf_epoch(c, 0.f, 0.f) != BMF_OK || bmf_sgd_timing(c, &ms, &l, 1) != BMF_OK)
        BMF_FAIL(BMF_E_DEVICE, "autotuner probe failed: " + c->err);
    return ms;
}

// Least-squares fit of T = c_r * crit + c_s * (b * cb * k) + c_f * b to the
// probes (non-negative coefficients; a negative one is dropped and the rest
// refitted).
Coef fit(const std::vector<std::array<double, 4>> &rows) {
    Coef c;
    std::vector<int> use = {0, 1, 2};
    for (int attempt = 0; attempt < 3; ++attempt) {
        const int d = (int)use.size();
        double A[3][3] = {{0}}, y[3] = {0};
        for (auto &r : rows)
            for (int a = 0; a < d; ++a) {
                y[a] += r[use[a]] * r[3];
                for (int bb = 0; bb < d; ++bb) A[a][bb] += r[use[a]] * r[use[bb]];
            }
        // Gaussian elimination
        double x[3] = {0};
        bool ok = true;
        for (int col = 0; col < d; ++col) {
            int piv = col;
            for (int rr = col + 1; rr < d; ++rr)
                if (std::fabs(A[rr][col]) > std::fabs(A[piv][col])) piv = rr;
            if (std::fabs(A[piv][col]) < 1e-300) {
                ok = false;
                break;
            }
            std::swap(A[piv], A[col]);
            std::swap(y[piv], y[col]);
            for (int rr = col + 1; rr < d; ++rr) {
                const double f = A[rr][col] / A[col][col];
                for (int cc = col; cc < d; ++cc) A[rr][cc] -= f * A[col][cc];
                y[rr] -= f * y[col];
            }
        }
        if (ok)
            for (int col = d - 1; col >= 0; --col) {
                double v = y[col];
                for (int cc = col + 1; cc < d; ++cc) v -= A[col][cc] * x[cc];
                x[col] = v / A[col][col];
            }
        int neg = -1;
        for (int a = 0; a < d; ++a)
            if (!ok || x[a] < 0) neg = a;
        if (neg < 0 || d == 1) {
            double out[3] = {0, 0, 0};
            for (int a = 0; a < d; ++a) out[use[a]] = std::max(0.0, x[a]);
            c.c_r = out[0] / 1e3;  // rows are in ms
            c.c_s = out[1] / 1e3;
            c.c_f = out[2] / 1e3;
            c.fitted = true;
            return c;
        }
        use.erase(use.begin() + neg);
    }
    return c;
}

std::vector<Candidate> candidates(int64_t m, int64_t n, int k, const int32_t *du, const int32_t *di, int64_t nnz,
                                  int device, hipStream_t s) {
    std::vector<Candidate> out;
    for (int b = 1; b <= 512; b *= 2) {
        if (!grid_ok(m, n, k, b, device)) continue;
        std::vector<int64_t> cnt;
        block_histogram(du, di, nnz, m, n, b, cnt, s);
        out.push_back({b, critical_path(cnt, b), (n + b - 1) / b});
    }
    return out;
}

template <class F>
bmf_status guarded_batch(bmf_batch *B, F &&f) {
    if (!B) return BMF_E_INVAL;
    if (B->poisoned) {
        B->err = "batch is poisoned by an earlier device error";
        return BMF_E_STATE;
    }
    try {
        BMF_HIP(hipSetDevice(B->device));
        f();
        return BMF_OK;
    } catch (const Error &e) {
        B->err = e.msg;
        if (e.code == BMF_E_DEVICE) B->poisoned = true;
        return e.code;
    } catch (const std::bad_alloc &) {
        B->err = "host allocation failed";
        return BMF_E_NOMEM;
    } catch (...) {
        B->err = "unexpected internal exception";
        B->poisoned = true;
        return BMF_E_DEVICE;
    }
}

void tune_and_load(bmf_batch *B) {
    // problems whose context does not exist yet: choose grids, then load
    std::vector<std::unique_ptr<Loaded>> *staged = &B->staged;
    const int np = (int)B->m.size();
    std::vector<int> todo;
    for (int p = 0; p < np; ++p)
        if (!B->probs[p] && (*staged)[p]) todo.push_back(p);
    if (todo.empty() && B->waves) return;
    const int k = B->k;
    // calibration on the largest staged (or loaded) problem
    Coef coef;
    const auto key = std::make_pair(B->device, k);
    {
        std::lock_guard<std::mutex> lk(g_coef_mu);
        if (g_coef.count(key)) coef = g_coef[key];
    }
    int big = -1;
    for (int p : todo)
        if (big < 0 || (*staged)[p]->nnz > (*staged)[big]->nnz) big = p;
    std::map<int, std::vector<Candidate>> cand;
    for (int p : todo) {
        const Loaded &L = *(*staged)[p];
        cand[p] = candidates(B->m[p], B->n[p], k, L.u.as<int32_t>(), L.i.as<int32_t>(), L.nnz, B->device, B->stream);
        if (cand[p].empty())
            BMF_FAIL(BMF_E_RANGE, "problem " + std::to_string(p) + ": no block grid fits the LDS item slice");
    }
    const bool need_auto = std::any_of(todo.begin(), todo.end(), [&](int p) { return B->b_req[p] <= 0; });
    if (big >= 0 && (need_auto || !B->waves) && (*staged)[big]->nnz > 0) {
        const Loaded &L = *(*staged)[big];
        auto &cs = cand[big];
        if (!coef.fitted && cs.size() >= 2) {
            // three grids spread over the feasible range
            std::vector<size_t> pick = {cs.size() - 1, cs.size() / 2, cs.size() >= 3 ? cs.size() - 3 : 0};
            std::sort(pick.begin(), pick.end());
            pick.erase(std::unique(pick.begin(), pick.end()), pick.end());
            std::vector<std::array<double, 4>> rows;
            for (size_t q : pick) {
                const Candidate &x = cs[q];
                const double ms = time_epoch(B->m[big], B->n[big], k, x.b, 4, L.u.as<int32_t>(), L.i.as<int32_t>(),
                                             L.r.as<float>(), L.nnz, B->stream);
                rows.push_back({(double)x.crit, (double)x.b * x.cb * k, (double)x.b, ms});
            }
            coef = fit(rows);
            std::lock_guard<std::mutex> lk(g_coef_mu);
            g_coef[key] = coef;
        }
        if (!B->waves) {
            // waves per workgroup: time both at the model's best grid
            const Candidate *best = &cs[0];
            for (auto &x : cs)
                if (model_ms(coef, x, k) < model_ms(coef, *best, k)) best = &x;
            const double t4 = time_epoch(B->m[big], B->n[big], k, best->b, 4, L.u.as<int32_t>(), L.i.as<int32_t>(),
                                         L.r.as<float>(), L.nnz, B->stream);
            const double t8 = time_epoch(B->m[big], B->n[big], k, best->b, 8, L.u.as<int32_t>(), L.i.as<int32_t>(),
                                         L.r.as<float>(), L.nnz, B->stream);
            B->waves = t8 < t4 ? 8 : 4;
        }
    }
    if (!B->waves) B->waves = 4;
    // per-problem grids: fastest by the model, then relax towards the
    // throughput bound
    std::map<int, const Candidate *> choice;
    for (int p : todo) {
        auto &cs = cand[p];
        if (B->b_req[p] > 0) {
            if (!grid_ok(B->m[p], B->n[p], k, B->b_req[p], B->device))
                BMF_FAIL(BMF_E_RANGE, "problem " + std::to_string(p) + ": grid " + std::to_string(B->b_req[p]) +
                                          " leaves an item slice too large for LDS");
            choice[p] = nullptr;
            continue;
        }
        const Candidate *best = &cs[0];
        for (auto &x : cs)
            if (model_ms(coef, x, k) < model_ms(coef, *best, k)) best = &x;
        choice[p] = best;
    }
    int cus = 0;
    BMF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
    for (int iter = 0; iter < 3; ++iter) {
        double total = 0, longest = 0;
        for (int p : todo)
            if (choice[p]) {
                total += work_ms(coef, *choice[p], k, (*staged)[p]->nnz);
                longest = std::max(longest, model_ms(coef, *choice[p], k));
            }
        const double bound = std::max(longest, total / std::max(1, cus));
        for (int p : todo) {
            if (!choice[p]) continue;
            for (auto &x : cand[p])  // smallest grid under the bound
                if (model_ms(coef, x, k) <= bound) {
                    choice[p] = &x;
                    break;
                }
        }
    }
    for (int p : todo) {
        const int b = choice[p] ? choice[p]->b : B->b_req[p];
        B->predicted_ms[p] = choice[p] ? model_ms(coef, *choice[p], k) : -1.0;
        bmf_ctx *c = nullptr;
        if (bmf_create(B->m[p], B->n[p], k, b, &c) != BMF_OK)
            BMF_FAIL(BMF_E_DEVICE, "problem " + std::to_string(p) + ": " + bmf_last_error(nullptr));
        std::unique_ptr<bmf_ctx, void (*)(bmf_ctx *)> guard(c, bmf_destroy);
        c->M.waves = B->waves;
        bmf_set_option(c, BMF_OPT_SEED, (int64_t)B->seed);
        bmf_set_option(c, BMF_OPT_ORDER_SEED, (int64_t)B->order_seed);
        bmf_set_option(c, BMF_OPT_STRATUM_ORDER, B->order_mode);
        const Loaded &L = *(*staged)[p];
        if (bmf_load_ratings_dev(c, L.u.as<int32_t>(), L.i.as<int32_t>(), L.r.as<float>(), L.nnz) != BMF_OK)
            BMF_FAIL(BMF_E_DEVICE, "problem " + std::to_string(p) + ": " + c->err);
        B->probs[p] = guard.release();
        (*staged)[p].reset();
    }
}

}  // namespace

extern "C" {

bmf_status bmf_batch_create(int32_t nprob, const int64_t *m, const int64_t *n, int32_t k, const int32_t *b,
                            bmf_batch **out) {
    if (!out || nprob < 1 || !m || !n || k < 1 || k > 128) return BMF_E_INVAL;
    *out = nullptr;
    for (int p = 0; p < nprob; ++p)
        if (m[p] < 1 || n[p] < 1 || m[p] >= INT32_MAX || n[p] >= INT32_MAX || (b && b[p] < 0)) return BMF_E_INVAL;
    bmf_batch *B = new (std::nothrow) bmf_batch();
    if (!B) return BMF_E_NOMEM;
    if (hipGetDevice(&B->device) != hipSuccess || hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
        delete B;
        return BMF_E_DEVICE;
    }
    B->k = k;
    B->m.assign(m, m + nprob);
    B->n.assign(n, n + nprob);
    B->b_req.assign(nprob, 0);
    if (b) B->b_req.assign(b, b + nprob);
    B->probs.assign(nprob, nullptr);
    B->predicted_ms.assign(nprob, -1.0);
    B->staged.resize(nprob);
    *out = B;
    return BMF_OK;
}

void bmf_batch_destroy(bmf_batch *B) {
    if (!B) return;
    (void)hipSetDevice(B->device);
    for (auto *c : B->probs) bmf_destroy(c);
    B->staged.clear();
    if (B->stream) {
        (void)hipStreamSynchronize(B->stream);
        (void)hipStreamDestroy(B->stream);
    }
    delete B;
}

const char *bmf_batch_last_error(const bmf_batch *B) { return B ? B->err.c_str() : ""; }

bmf_status bmf_batch_set_option(bmf_batch *B, int32_t key, int64_t value) {
    return guarded_batch(B, [&] {
        for (auto *c : B->probs)
            if (c) BMF_FAIL(BMF_E_STATE, "batch options must be set before any problem is loaded");
        switch (key) {
        case BMF_OPT_SEED: B->seed = (uint64_t)value; break;
        case BMF_OPT_ORDER_SEED: B->order_seed = (uint64_t)value; break;
        case BMF_OPT_STRATUM_ORDER:
            if (value != 0 && value != 1) BMF_FAIL(BMF_E_INVAL, "stratum order must be 0 or 1");
            B->order_mode = (int)value;
            break;
        case BMF_OPT_WAVES_PER_BLOCK:
            if (value != 0 && value != 4 && value != 8) BMF_FAIL(BMF_E_INVAL, "waves per block must be 0, 4 or 8");
            B->waves = (int)value;
            break;
        default: BMF_FAIL(BMF_E_INVAL, "option not supported on a batch");
        }
    });
}

bmf_status bmf_batch_load(bmf_batch *B, int32_t p, const int32_t *u, const int32_t *i, const float *r, int64_t nnz) {
    return guarded_batch(B, [&] {
        if (p < 0 || p >= (int)B->m.size()) BMF_FAIL(BMF_E_INVAL, "problem index out of range");
        if (B->probs[p]) BMF_FAIL(BMF_E_STATE, "problem already loaded");
        if (nnz < 0 || (nnz > 0 && (!u || !i || !r))) BMF_FAIL(BMF_E_INVAL, "bad rating arrays");
        auto L = std::make_unique<Loaded>();
        L->nnz = nnz;
        L->u.alloc(nnz * 4);
        L->i.alloc(nnz * 4);
        L->r.alloc(nnz * 4);
        if (nnz) {
            BMF_HIP(hipMemcpyAsync(L->u.p, u, nnz * 4, hipMemcpyHostToDevice, B->stream));
            BMF_HIP(hipMemcpyAsync(L->i.p, i, nnz * 4, hipMemcpyHostToDevice, B->stream));
            BMF_HIP(hipMemcpyAsync(L->r.p, r, nnz * 4, hipMemcpyHostToDevice, B->stream));
        }
        DevBuf scratch;
        const int64_t bad = validate_coo(L->u.as<int32_t>(), L->i.as<int32_t>(), L->r.as<float>(), nnz, B->m[p],
                                         B->n[p], scratch, B->stream);
        if (bad >= 0) BMF_FAIL(BMF_E_RANGE, "problem " + std::to_string(p) + ": rating " + std::to_string(bad) +
                                                " is out of range or not finite");
        B->staged[p] = std::move(L);
    });
}

bmf_status bmf_batch_tune(bmf_batch *B) {
    return guarded_batch(B, [&] { tune_and_load(B); });
}

bmf_status bmf_batch_epochs(bmf_batch *B, int32_t epochs, const float hp[8]) {
    return guarded_batch(B, [&] {
        if (epochs < 1 || !hp) BMF_FAIL(BMF_E_INVAL, "epochs must be >= 1 and hp non-null");
        for (int q = 0; q < 8; ++q)
            if (!std::isfinite(hp[q])) BMF_FAIL(BMF_E_INVAL, "non-finite hyper-parameter");
        tune_and_load(B);
        const int np = (int)B->m.size();
        for (int p = 0; p < np; ++p)
            if (!B->probs[p]) BMF_FAIL(BMF_E_STATE, "problem " + std::to_string(p) + " not loaded");
        // problem table
        std::vector<BatchProblem> tab(np);
        const size_t tab_bytes = np * sizeof(BatchProblem);
        if (B->d_probs.bytes < tab_bytes) B->d_probs.alloc(tab_bytes);
        size_t lds = 0;
        for (int p = 0; p < np; ++p) {
            Model &M = B->probs[p]->M;
            ensure_plan(M);
            if (!M.plan.ok) BMF_FAIL(BMF_E_STATE, "problem " + std::to_string(p) + " has no plan for the LDS kernel");
            tab[p] = BatchProblem{M.plan.steps.as<SlotRec>(), M.plan.blk_step.as<int64_t>(), M.P.as<float>(),
                                  M.Q.as<float>(), M.bu.as<float>(), M.bi.as<float>(), M.n, M.part.rb, M.part.cb,
                                  (float)M.mu, M.b, M.plan.S, M.plan.CH};
            lds = std::max(lds, plan_lds(M.plan.kp, M.part.cb, M.plan.S, M.plan.CH).total);
        }
        // work list, position-major: the items of position t are contiguous
        int64_t maxT = 0;
        for (int p = 0; p < np; ++p) maxT = std::max(maxT, (int64_t)epochs * B->probs[p]->M.b);
        std::vector<BatchItem> items;
        std::vector<int64_t> first(maxT + 1, 0);
        std::vector<std::vector<int32_t>> order(np);
        for (int64_t t = 0; t < maxT; ++t) {
            first[t] = (int64_t)items.size();
            for (int p = 0; p < np; ++p) {
                Model &M = B->probs[p]->M;
                if (t >= (int64_t)epochs * M.b) continue;
                const int pos = (int)(t % M.b);
                if (pos == 0) {
                    order[p].resize(M.b);
                    schedule(M.b, M.order_seed, M.epoch + (int)(t / M.b), M.order_mode, order[p].data());
                }
                for (int j = 0; j < M.b; ++j) items.push_back(BatchItem{p, (int32_t)t, order[p][pos], j});
            }
        }
        first[maxT] = (int64_t)items.size();
        if (B->d_items.bytes < items.size() * sizeof(BatchItem)) B->d_items.alloc(items.size() * sizeof(BatchItem));
        BMF_HIP(hipMemcpyAsync(B->d_probs.p, tab.data(), tab_bytes, hipMemcpyHostToDevice, B->stream));
        BMF_HIP(hipMemcpyAsync(B->d_items.p, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                               B->stream));
        // the factor tables are touched by the batch stream only after the
        // problems' own streams are idle
        for (int p = 0; p < np; ++p) BMF_HIP(hipStreamSynchronize(B->probs[p]->M.stream));
        // timing events, destroyed on every way out
        struct Events {
            hipEvent_t a = nullptr, b = nullptr;
            ~Events() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev;
        BMF_HIP(hipEventCreate(&ev.a));
        BMF_HIP(hipEventCreate(&ev.b));
        const hipEvent_t e0 = ev.a, e1 = ev.b;
        BMF_HIP(hipEventRecord(e0, B->stream));
        const HP h{hp[0], hp[1], hp[2], hp[3], hp[4], hp[5], hp[6], hp[7]};
        for (int64_t t = 0; t < maxT; ++t)
            sgd_positions_launch(B->k, B->waves, B->d_probs.as<BatchProblem>(), B->d_items.as<BatchItem>() + first[t],
                                 first[t + 1] - first[t], h, lds, B->stream);
        BMF_HIP(hipEventRecord(e1, B->stream));
        BMF_HIP(hipStreamSynchronize(B->stream));
        float ms = 0;
        BMF_HIP(hipEventElapsedTime(&ms, e0, e1));
        B->ms += ms;
        B->launches += maxT;
        for (int p = 0; p < np; ++p) {
            B->probs[p]->M.epoch += epochs;
            B->probs[p]->M.bf16_valid = false;
        }
    });
}

bmf_status bmf_batch_problem(bmf_batch *B, int32_t p, bmf_ctx **out) {
    return guarded_batch(B, [&] {
        if (!out || p < 0 || p >= (int)B->m.size()) BMF_FAIL(BMF_E_INVAL, "bad problem index");
        tune_and_load(B);
        if (!B->probs[p]) BMF_FAIL(BMF_E_STATE, "problem not loaded");
        *out = B->probs[p];
    });
}

bmf_status bmf_batch_info(bmf_batch *B, int32_t p, int32_t *b_out, int32_t *waves_out, double *predicted_ms) {
    return guarded_batch(B, [&] {
        if (p < 0 || p >= (int)B->m.size()) BMF_FAIL(BMF_E_INVAL, "bad problem index");
        tune_and_load(B);
        if (b_out) *b_out = B->probs[p] ? B->probs[p]->M.b : 0;
        if (waves_out) *waves_out = B->waves;
        if (predicted_ms) *predicted_ms = B->predicted_ms[p];
    });
}

bmf_status bmf_batch_timing(bmf_batch *B, double *ms, int64_t *launches, int32_t reset) {
    return guarded_batch(B, [&] {
        if (ms) *ms = B->ms;
        if (launches) *launches = B->launches;
        if (reset) {
            B->ms = 0;
            B->launches = 0;
        }
    });
}

}  // extern "C"
