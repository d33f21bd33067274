// Serving: continuous batching of top-K recommendation requests and new-user
// fold-in requests (folding-in, Section 2.1 and Section 6) on a trained
// model.
//
// A scheduler thread owns the device work.  Submitted requests wait in a
// FIFO queue.  The device workspace (the memory budget) is split into one
// partition per batch slot; whenever a slot is free the scheduler forms a
// batch from the head of the queue, taking requests while their workspace
// fits the partition (admission by memory) and the row cap allows, and
// enqueues it on the slot's stream: uploads, fold-in kernel for the batch's
// new users, user-row gather, one scoring pass per precision over all rows
// of the batch, downloads, completion event.  When the event has fired, a
// completion thread copies the results out of the slot's pinned staging and
// frees the slot, so the scheduler goes on launching meanwhile.  Requests
// that arrive while batches are on the GPU go into the next batch; batches
// on different slots overlap on the device.  Every row is scored on its own (the MFMA
// latent order is fixed and the selection is exact with a fixed tie rule),
// so a request's result does not depend on the batch it lands in.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"

using namespace bmf;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    int64_t id = 0;
    bool foldin = false;
    int precision = 0, K = 0;
    std::vector<int32_t> users, items;
    std::vector<float> ratings;
    Clock::time_point t_submit, t_done;
    bool done = false;
    // results, written once by a completion thread (no zero fill first)
    std::unique_ptr<int32_t[]> out_items;
    std::unique_ptr<float[]> out_scores;
    size_t out_n = 0;
    std::vector<float> out_p;
    float out_bu = 0.f;
    size_t bytes = 0;
};

// Where one request's rows sit inside a batch.
struct Placement {
    std::shared_ptr<Request> req;
    int group;      // precision
    int64_t row;    // first row in the group
};

struct Group {
    int64_t nusers = 0, nfold = 0, fold_ratings = 0;
    int K = 0, max_nr = 0;
    TopkPlan plan;
    size_t off_in = 0, off_buf = 0, off_work = 0, off_items = 0, off_scores = 0, total = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char *dev = nullptr;   // partition of the device workspace
    unsigned char *hin = nullptr;   // pinned staging for inputs
    unsigned char *hout = nullptr;  // pinned staging for outputs
    bool busy = false;       // a batch is in flight or its results are being copied out
    bool finishing = false;  // handed to a completion thread
    std::vector<Placement> placed;
    Group g[2];
    size_t host_off_out[2] = {0, 0};
    size_t bytes = 0;
};

}  // namespace

struct bmf_server {
    bmf_ctx *ctx = nullptr;
    bmf_server_config cfg{};
    size_t part_bytes = 0;
    DevBuf arena;
    std::vector<Slot> slots;
    mutable std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> live;
    int64_t next_id = 1;
    bool stop = false, failed = false;
    std::string err;
    std::thread worker;
    // completion threads: copy finished batches' results out of the pinned
    // staging while the scheduler keeps launching
    std::vector<std::thread> finishers;
    std::deque<int> finished;  // slots whose batch completed on the device
    std::condition_variable fcv;
    bool finishers_stop = false;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, rows = 0;
    size_t bytes_in_use = 0, peak_bytes = 0;
    std::vector<double> lat_ms;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t group_bytes(Model &M, int64_t nusers, int64_t nfold, int64_t fold_ratings, int K, int precision, int Kc) {
    Group G;
    G.nusers = nusers;
    G.nfold = nfold;
    G.fold_ratings = fold_ratings;
    G.K = K;
    const TopkPlan T = topk_plan(M, nusers + nfold, K, precision, Kc);
    size_t o = align256(std::max<int64_t>(nusers, 1) * 4) + 2 * align256(std::max<int64_t>(fold_ratings, 1) * 4) +
               align256((nfold + 1) * 8) + align256(std::max<int64_t>(nfold, 1) * 4);
    o += align256(T.total);
    o += 2 * align256((size_t)(nusers + nfold) * K * 4);
    return o;
}

size_t request_bytes(Model &M, const Request &r, int Kc) {
    return group_bytes(M, r.foldin ? 0 : (int64_t)r.users.size(), r.foldin ? 1 : 0,
                       r.foldin ? (int64_t)r.items.size() : 0, r.K, r.precision, Kc);
}

// Host staging bytes of a request: inputs (ids, ratings, offsets) and
// outputs (items, scores, folded-in vector and bias).
size_t request_host_in(const Request &r) { return align256(r.users.size() * 4 + r.items.size() * 8 + 64); }
size_t request_host_out(const Request &r, int k) {
    const size_t rows = r.foldin ? 1 : r.users.size();
    const size_t kp = (size_t)(k + 15) / 16 * 16;
    return align256(rows * r.K * 8 + (r.foldin ? (kp + 1) * 4 : 0));
}

void launch_batch(bmf_server *S, Slot &sl) {
    Model &M = S->ctx->M;
    const int k = M.k;
    const int Kc = S->cfg.Kc;
    // group sizes
    for (int g = 0; g < 2; ++g) sl.g[g] = Group{};
    for (auto &pl : sl.placed) {
        Group &G = sl.g[pl.group];
        if (pl.req->foldin) {
            G.nfold += 1;
            G.fold_ratings += (int64_t)pl.req->items.size();
            G.max_nr = std::max<int>(G.max_nr, (int)pl.req->items.size());
        } else {
            G.nusers += (int64_t)pl.req->users.size();
        }
        G.K = std::max(G.K, pl.req->K);
    }
    // rows: top-K users first, then folded-in users
    {
        int64_t urow[2] = {0, 0}, frow[2] = {sl.g[0].nusers, sl.g[1].nusers};
        for (auto &pl : sl.placed) {
            if (pl.req->foldin)
                pl.row = frow[pl.group]++;
            else {
                pl.row = urow[pl.group];
                urow[pl.group] += (int64_t)pl.req->users.size();
            }
        }
    }
    size_t dev_off = 0, hin_off = 0, hout_off = 0;
    for (int g = 0; g < 2; ++g) {
        Group &G = sl.g[g];
        const int64_t rows = G.nusers + G.nfold;
        if (rows == 0) continue;
        G.plan = topk_plan(M, rows, G.K, g, Kc);
        size_t o = dev_off;
        auto take = [&](size_t b) {
            size_t at = o;
            o += align256(b);
            return at;
        };
        // inputs laid out as in the pinned staging, so one copy moves them:
        // users | fold-in items | ratings, then (256-byte aligned) offsets
        const size_t in_lists = align256((size_t)(G.nusers + 2 * G.fold_ratings) * 4);
        const size_t in_bytes = in_lists + (size_t)(G.nfold + 1) * 8;
        G.off_in = take(in_bytes);
        G.off_buf = take(std::max<int64_t>(G.nfold, 1) * 4);
        G.off_work = take(G.plan.total);
        G.off_items = take((size_t)rows * G.K * 4);
        G.off_scores = take((size_t)rows * G.K * 4);  // right after the items, as in the staging
        if (o > S->part_bytes) BMF_FAIL(BMF_E_DEVICE, "internal: batch workspace exceeds its partition");
        dev_off = o;
        // host inputs: users | fold-in items | ratings | offsets, one copy
        unsigned char *h = sl.hin + hin_off;
        int32_t *hu = reinterpret_cast<int32_t *>(h);
        int32_t *hi = hu + G.nusers;
        float *hr = reinterpret_cast<float *>(hi + G.fold_ratings);
        int64_t *hoff = reinterpret_cast<int64_t *>(h + in_lists);  // hin_off is a multiple of 256
        int64_t fo = 0, fi = 0;
        for (auto &pl : sl.placed) {
            if (pl.group != g) continue;
            if (pl.req->foldin) {
                std::memcpy(hi + fo, pl.req->items.data(), pl.req->items.size() * 4);
                std::memcpy(hr + fo, pl.req->ratings.data(), pl.req->ratings.size() * 4);
                hoff[fi] = fo;
                fo += (int64_t)pl.req->items.size();
                ++fi;
            } else {
                std::memcpy(hu + pl.row, pl.req->users.data(), pl.req->users.size() * 4);
            }
        }
        hoff[fi] = fo;
        unsigned char *d = sl.dev;
        const hipStream_t st = sl.stream;
        unsigned char *din = d + G.off_in;
        BMF_HIP(hipMemcpyAsync(din, h, in_bytes, hipMemcpyHostToDevice, st));
        const int32_t *d_users = reinterpret_cast<const int32_t *>(din);
        const int32_t *d_fitems = d_users + G.nusers;
        const float *d_fr = reinterpret_cast<const float *>(d_fitems + G.fold_ratings);
        const int64_t *d_foff = reinterpret_cast<const int64_t *>(din + in_lists);
        hin_off += align256(in_bytes);
        // user rows: gather (rows past nusers become zero rows), then the
        // folded-in users overwrite their rows
        unsigned char *work = d + G.off_work;
        {
            // ids are read for the first nusers rows only; every later row
            // (folded-in users, padding) starts as a zero row
            TopkPlan P2 = G.plan;
            P2.nu = G.nusers;
            topk_gather(M, P2, d_users, work, st);
        }
        if (G.nfold) {
            const HP hp{S->cfg.foldin_lr, S->cfg.foldin_reg, 0.f, 0.f, S->cfg.foldin_lr, S->cfg.foldin_reg, 0.f, 0.f};
            float *Ug = reinterpret_cast<float *>(work + G.plan.off_ug) + G.nusers * G.plan.kp;
            uint16_t *Ugb = g == 1 ? reinterpret_cast<uint16_t *>(work + G.plan.off_ugb) + G.nusers * G.plan.kb : nullptr;
            float *ub = reinterpret_cast<float *>(work + G.plan.off_ub) + G.nusers;
            float *bu_f = reinterpret_cast<float *>(d + G.off_buf);
            foldin_launch(M, d_fitems, d_fr, d_foff, G.nfold, G.max_nr, S->cfg.foldin_passes, hp, Ug, G.plan.kp,
                          bu_f, st);
            foldin_rows(bu_f, G.nfold, (float)M.mu, k, G.plan.kp, G.plan.kb, Ug, Ugb, ub, st);
        }
        int32_t *ditems = reinterpret_cast<int32_t *>(d + G.off_items);
        float *dscores = reinterpret_cast<float *>(d + G.off_scores);
        topk_score(M, G.plan, work, ditems, dscores, st);
        // outputs: items and scores (adjacent on both sides) in one copy
        sl.host_off_out[g] = hout_off;
        const size_t list_bytes = align256((size_t)rows * G.K * 4);
        if (G.off_scores != G.off_items + list_bytes)
            BMF_FAIL(BMF_E_DEVICE, "internal: result lists are not adjacent in the workspace");
        BMF_HIP(hipMemcpyAsync(sl.hout + hout_off, ditems, list_bytes + (size_t)rows * G.K * 4, hipMemcpyDeviceToHost,
                               st));
        hout_off += 2 * list_bytes;
        if (G.nfold) {
            BMF_HIP(hipMemcpyAsync(sl.hout + hout_off, work + G.plan.off_ug + (size_t)G.nusers * G.plan.kp * 4,
                                   (size_t)G.nfold * G.plan.kp * 4, hipMemcpyDeviceToHost, st));
            hout_off += align256((size_t)G.nfold * G.plan.kp * 4);
            BMF_HIP(hipMemcpyAsync(sl.hout + hout_off, d + G.off_buf, (size_t)G.nfold * 4, hipMemcpyDeviceToHost, st));
            hout_off += align256((size_t)G.nfold * 4);
        }
    }
    BMF_HIP(hipEventRecord(sl.done, sl.stream));
}

// Copies a completed batch's results from the slot's pinned staging into
// its requests (no lock: until published, the slot and its requests are the
// caller's alone).
void copy_results(bmf_server *S, Slot &sl) {
    const int k = S->ctx->M.k;
    for (int g = 0; g < 2; ++g) {
        Group &G = sl.g[g];
        const int64_t rows = G.nusers + G.nfold;
        if (rows == 0) continue;
        const unsigned char *h = sl.hout + sl.host_off_out[g];
        const int32_t *it = reinterpret_cast<const int32_t *>(h);
        const float *sc = reinterpret_cast<const float *>(h + align256((size_t)rows * G.K * 4));
        const float *pv = reinterpret_cast<const float *>(h + 2 * align256((size_t)rows * G.K * 4));
        const float *bv = reinterpret_cast<const float *>(reinterpret_cast<const unsigned char *>(pv) +
                                                          align256((size_t)G.nfold * G.plan.kp * 4));
        for (auto &pl : sl.placed) {
            if (pl.group != g) continue;
            Request &r = *pl.req;
            const int64_t nrow = r.foldin ? 1 : (int64_t)r.users.size();
            r.out_n = (size_t)nrow * r.K;
            r.out_items.reset(new int32_t[r.out_n]);
            r.out_scores.reset(new float[r.out_n]);
            if (r.K == G.K) {
                std::memcpy(r.out_items.get(), it + pl.row * G.K, r.out_n * 4);
                std::memcpy(r.out_scores.get(), sc + pl.row * G.K, r.out_n * 4);
            } else {
                for (int64_t q = 0; q < nrow; ++q) {
                    std::memcpy(&r.out_items[q * r.K], it + (pl.row + q) * G.K, r.K * 4);
                    std::memcpy(&r.out_scores[q * r.K], sc + (pl.row + q) * G.K, r.K * 4);
                }
            }
            if (r.foldin) {
                const int64_t fidx = pl.row - G.nusers;
                r.out_p.assign(pv + fidx * G.plan.kp, pv + fidx * G.plan.kp + k);
                r.out_bu = bv[fidx];
            }
        }
    }
}

// Marks a copied batch's requests done and frees its slot (lock held).
void publish_batch(bmf_server *S, Slot &sl) {
    const auto now = Clock::now();
    for (auto &pl : sl.placed) {
        Request &r = *pl.req;
        r.t_done = now;
        r.done = true;
        S->completed += 1;
        S->lat_ms.push_back(std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count());
    }
    S->bytes_in_use -= sl.bytes;
    sl.bytes = 0;
    sl.placed.clear();
    sl.finishing = false;
    sl.busy = false;
}

void finisher(bmf_server *S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->fcv.wait(lk, [&] { return S->finishers_stop || !S->finished.empty(); });
        if (S->finished.empty()) break;  // stop, nothing left
        Slot &sl = S->slots[S->finished.front()];
        S->finished.pop_front();
        bool ok = true;
        {
            lk.unlock();
            try {
                copy_results(S, sl);
            } catch (...) {
                ok = false;
            }
            lk.lock();
        }
        if (ok) {
            publish_batch(S, sl);
        } else {
            // the server stops: pollers of these requests get the failure,
            // and the slot is let go so that the scheduler can end
            S->failed = true;
            S->err = "server failed: host allocation for results failed";
            S->bytes_in_use -= sl.bytes;
            sl.bytes = 0;
            sl.placed.clear();
            sl.finishing = false;
            sl.busy = false;
        }
        S->cv.notify_all();
    }
}

// Releases a held lock for a scope and takes it back on exit (also when an
// exception leaves the scope).
struct UnlockGuard {
    std::unique_lock<std::mutex> &lk;
    explicit UnlockGuard(std::unique_lock<std::mutex> &l) : lk(l) { lk.unlock(); }
    ~UnlockGuard() { lk.lock(); }
};

void scheduler(bmf_server *S) {
    std::unique_lock<std::mutex> lk(S->mu);
    try {
        BMF_HIP(hipSetDevice(S->ctx->M.device));
        Model &M = S->ctx->M;
        while (true) {
            if (S->failed) break;  // a completion thread failed
            bool progressed = false;
            // completions
            for (size_t q = 0; q < S->slots.size(); ++q) {
                Slot &sl = S->slots[q];
                if (!sl.busy || sl.finishing) continue;
                const hipError_t e = hipEventQuery(sl.done);
                if (e == hipSuccess) {
                    sl.finishing = true;
                    S->finished.push_back((int)q);
                    progressed = true;
                } else if (e != hipErrorNotReady) {
                    BMF_HIP(e);
                }
            }
            if (progressed) S->fcv.notify_all();
            // new batches
            for (auto &sl : S->slots) {
                if (sl.busy || S->queue.empty()) continue;
                size_t bytes_dev = 0, bytes_in = 4096, bytes_out = 4096;
                int64_t rows = 0;
                int64_t n_req = 0;
                // per-group accumulators for the exact workspace of the batch
                int64_t gu[2] = {0, 0}, gf[2] = {0, 0}, gr[2] = {0, 0};
                int gk[2] = {0, 0};
                while (!S->queue.empty()) {
                    auto &r = S->queue.front();
                    const int g = r->precision;
                    int64_t u2[2] = {gu[0], gu[1]}, f2[2] = {gf[0], gf[1]}, r2[2] = {gr[0], gr[1]};
                    int k2[2] = {gk[0], gk[1]};
                    if (r->foldin) {
                        f2[g] += 1;
                        r2[g] += (int64_t)r->items.size();
                    } else {
                        u2[g] += (int64_t)r->users.size();
                    }
                    k2[g] = std::max(k2[g], r->K);
                    size_t need = 0;
                    for (int q = 0; q < 2; ++q)
                        if (u2[q] + f2[q] > 0) need += group_bytes(M, u2[q], f2[q], r2[q], k2[q], q, S->cfg.Kc);
                    const size_t hin = bytes_in + request_host_in(*r), hout = bytes_out + request_host_out(*r, M.k);
                    const int64_t nrows = rows + (r->foldin ? 1 : (int64_t)r->users.size());
                    const bool cap_ok = n_req == 0 || (nrows <= S->cfg.max_batch_rows &&
                                                       (S->cfg.max_requests_per_batch <= 0 ||
                                                        n_req < S->cfg.max_requests_per_batch));
                    if (need > S->part_bytes || hin > S->part_bytes || hout > S->part_bytes || !cap_ok) break;
                    bytes_dev = need;
                    bytes_in = hin;
                    bytes_out = hout;
                    rows = nrows;
                    for (int q = 0; q < 2; ++q) {
                        gu[q] = u2[q];
                        gf[q] = f2[q];
                        gr[q] = r2[q];
                        gk[q] = k2[q];
                    }
                    sl.placed.push_back(Placement{r, g, 0});
                    S->queue.pop_front();
                    ++n_req;
                }
                if (sl.placed.empty()) continue;
                sl.bytes = bytes_dev;
                S->bytes_in_use += bytes_dev;
                S->peak_bytes = std::max(S->peak_bytes, S->bytes_in_use);
                S->batches += 1;
                S->rows += rows;
                // busy before the lock is released, so that a drain never sees
                // the batch's requests neither queued nor in a busy slot
                sl.busy = true;
                {
                    // the slot and its requests are the scheduler's alone now:
                    // submissions and polls go on while the batch is launched
                    UnlockGuard ug(lk);
                    launch_batch(S, sl);
                }
                progressed = true;
            }
            if (S->stop && S->queue.empty()) {
                bool any = false;
                for (auto &sl : S->slots) any |= sl.busy;
                if (!any) break;
            }
            if (!progressed) {
                bool any_busy = false;
                for (auto &sl : S->slots) any_busy |= sl.busy;
                if (any_busy) {
                    lk.unlock();
                    std::this_thread::yield();
                    lk.lock();
                } else {
                    S->cv.wait_for(lk, std::chrono::milliseconds(2));
                }
            }
        }
    } catch (const Error &e) {
        S->failed = true;
        S->err = "server failed: " + e.msg;
        S->ctx->poisoned = e.code == BMF_E_DEVICE;
    } catch (...) {
        S->failed = true;
        S->err = "server failed: unexpected exception in the serving scheduler";
    }
    S->cv.notify_all();
}

template <class F>
bmf_status guarded_server(bmf_server *S, F &&f) {
    if (!S) return BMF_E_INVAL;
    try {
        f();
        return BMF_OK;
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        return BMF_E_NOMEM;
    }
}

bmf_status submit(bmf_server *S, std::shared_ptr<Request> r, int64_t *id) {
    const Clock::time_point t0 = Clock::now();  // latency counts from the call, including any wait for the queue
    return guarded_server(S, [&] {
        if (!id) BMF_FAIL(BMF_E_INVAL, "null id");
        Model &M = S->ctx->M;
        if (r->K < 1 || r->K > 512) BMF_FAIL(BMF_E_INVAL, "K must be in [1, 512]");
        if (r->precision != 0 && r->precision != 1) BMF_FAIL(BMF_E_INVAL, "precision must be 0 or 1");
        if (r->precision == 1) {
            const int kc = topk_candidates(r->K, S->cfg.Kc);
            if (kc > 1008) BMF_FAIL(BMF_E_INVAL, "BF16 candidates per user must be at most 1008");
        }
        for (int32_t u : r->users)
            if (u < 0 || u >= M.m) BMF_FAIL(BMF_E_RANGE, "user id out of range");
        for (size_t t = 0; t < r->items.size(); ++t)
            if (r->items[t] < 0 || r->items[t] >= M.n || !std::isfinite(r->ratings[t]))
                BMF_FAIL(BMF_E_RANGE, "fold-in rating out of range");
        const size_t need = request_bytes(M, *r, S->cfg.Kc);
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->failed) BMF_FAIL(BMF_E_DEVICE, S->err);
        if (need > S->part_bytes || request_host_in(*r) + 4096 > S->part_bytes ||
            request_host_out(*r, M.k) + 4096 > S->part_bytes) {
            S->rejected += 1;
            BMF_FAIL(BMF_E_NOMEM, "request needs " + std::to_string(need) + " bytes of workspace; a batch has " +
                                      std::to_string(S->part_bytes));
        }
        r->id = S->next_id++;
        r->t_submit = t0;
        S->live[r->id] = r;
        S->queue.push_back(r);
        S->submitted += 1;
        *id = r->id;
        S->cv.notify_all();
    });
}

}  // namespace

extern "C" {

bmf_status bmf_server_create(bmf_ctx *c, const bmf_server_config *cfg, bmf_server **out) {
    if (!c || !out) return BMF_E_INVAL;
    *out = nullptr;
    if (c->poisoned) return BMF_E_STATE;
    auto S = std::make_unique<bmf_server>();
    S->ctx = c;
    bmf_server_config d{};
    if (cfg) d = *cfg;
    if (d.mem_budget_bytes <= 0) d.mem_budget_bytes = (int64_t)1 << 30;
    // defaults measured on the serving workload (1M x 100k, k = 128): four
    // batches of up to 4,096 rows in flight gave the highest saturated rate
    if (d.max_batches <= 0) d.max_batches = 4;
    if (d.max_batches > 4) d.max_batches = 4;
    if (d.max_batch_rows <= 0) d.max_batch_rows = 4096;
    if (d.foldin_passes <= 0) d.foldin_passes = 10;
    if (d.foldin_lr <= 0.f) d.foldin_lr = 0.005f;
    if (d.foldin_reg <= 0.f) d.foldin_reg = 0.05f;
    if (d.Kc < 0 || d.Kc > 1008) return BMF_E_INVAL;  // the selection kernels hold at most 1008 candidates
    S->cfg = d;
    try {
        Model &M = c->M;
        BMF_HIP(hipSetDevice(M.device));
        if (M.k > 256) BMF_FAIL(BMF_E_INVAL, "serving supports k <= 256");
        ensure_bf16_items(M, true);
        BMF_HIP(hipStreamSynchronize(M.stream));
        S->part_bytes = ((size_t)d.mem_budget_bytes / d.max_batches) & ~size_t(255);
        S->arena.alloc(S->part_bytes * d.max_batches);
        S->slots.resize(d.max_batches);
        for (int q = 0; q < d.max_batches; ++q) {
            Slot &sl = S->slots[q];
            BMF_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            BMF_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
            sl.dev = S->arena.as<unsigned char>() + q * S->part_bytes;
            BMF_HIP(hipHostMalloc((void **)&sl.hin, S->part_bytes, hipHostMallocDefault));
            BMF_HIP(hipHostMalloc((void **)&sl.hout, S->part_bytes, hipHostMallocDefault));
        }
    } catch (const Error &e) {
        c->err = e.msg;
        for (auto &sl : S->slots) {
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.hin) (void)hipHostFree(sl.hin);
            if (sl.hout) (void)hipHostFree(sl.hout);
        }
        return e.code;
    }
    bmf_server *raw = S.release();
    for (int q = 0; q < 2; ++q) raw->finishers.emplace_back(finisher, raw);
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return BMF_OK;
}

void bmf_server_destroy(bmf_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->queue.clear();
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    {
        // the scheduler has handed over every completed batch
        std::lock_guard<std::mutex> lk(S->mu);
        S->finishers_stop = true;
    }
    S->fcv.notify_all();
    for (auto &t : S->finishers)
        if (t.joinable()) t.join();
    (void)hipSetDevice(S->ctx->M.device);
    for (auto &sl : S->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.hin) (void)hipHostFree(sl.hin);
        if (sl.hout) (void)hipHostFree(sl.hout);
    }
    delete S;
}

const char *bmf_server_last_error(const bmf_server *S) {
    // a copy per calling thread: the scheduler thread may set the message
    thread_local std::string msg;
    if (!S) return "";
    std::lock_guard<std::mutex> lk(S->mu);
    msg = S->err;
    return msg.c_str();
}

bmf_status bmf_server_submit_topk(bmf_server *S, const int32_t *users, int32_t nu, int32_t K, int32_t precision,
                                  int64_t *id) {
    if (!S || !users || nu < 1) return BMF_E_INVAL;
    auto r = std::make_shared<Request>();
    r->users.assign(users, users + nu);
    r->K = K;
    r->precision = precision;
    return submit(S, r, id);
}

bmf_status bmf_server_submit_foldin(bmf_server *S, const int32_t *items, const float *ratings, int32_t nr, int32_t K,
                                    int32_t precision, int64_t *id) {
    if (!S || !items || !ratings || nr < 1) return BMF_E_INVAL;
    auto r = std::make_shared<Request>();
    r->foldin = true;
    r->items.assign(items, items + nr);
    r->ratings.assign(ratings, ratings + nr);
    r->K = K;
    r->precision = precision;
    return submit(S, r, id);
}

bmf_status bmf_server_poll(bmf_server *S, int64_t id, int32_t wait, int32_t *done, int32_t *items_out,
                           float *scores_out, float *p_out, float *bu_out, int64_t *latency_ns) {
    if (!S || !done) return BMF_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto itr = S->live.find(id);
    if (itr == S->live.end()) {
        S->err = "unknown request id";
        return BMF_E_INVAL;
    }
    auto r = itr->second;
    if (wait)
        S->cv.wait(lk, [&] { return r->done || S->failed; });
    if (!r->done) {
        *done = 0;
        return S->failed ? BMF_E_DEVICE : BMF_OK;  // the scheduler's message stays in err
    }
    *done = 1;
    if (items_out) std::memcpy(items_out, r->out_items.get(), r->out_n * 4);
    if (scores_out) std::memcpy(scores_out, r->out_scores.get(), r->out_n * 4);
    if (p_out && r->foldin) std::memcpy(p_out, r->out_p.data(), r->out_p.size() * 4);
    if (bu_out && r->foldin) *bu_out = r->out_bu;
    if (latency_ns)
        *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(r->t_done - r->t_submit).count();
    S->live.erase(itr);
    return BMF_OK;
}

bmf_status bmf_server_drain(bmf_server *S) {
    if (!S) return BMF_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] {
        if (S->failed) return true;
        if (!S->queue.empty()) return false;
        for (auto &sl : S->slots)
            if (sl.busy) return false;
        return true;
    });
    return S->failed ? BMF_E_DEVICE : BMF_OK;
}

bmf_status bmf_server_get_stats(bmf_server *S, bmf_server_stats *out, int32_t reset) {
    if (!S || !out) return BMF_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    bmf_server_stats st{};
    st.submitted = S->submitted;
    st.completed = S->completed;
    st.rejected = S->rejected;
    st.batches = S->batches;
    st.rows = S->rows;
    st.budget_bytes = (int64_t)(S->part_bytes * S->slots.size());
    st.peak_bytes = (int64_t)S->peak_bytes;
    st.queue_depth = (int64_t)S->queue.size();
    std::vector<double> v = S->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = std::min(v.size() - 1, (size_t)std::ceil(p * (double)v.size()) - (p > 0 ? 1 : 0));
            return v[i];
        };
        st.p50_ms = pct(0.50);
        st.p90_ms = pct(0.90);
        st.p99_ms = pct(0.99);
        st.max_ms = v.back();
        double s = 0;
        for (double x : v) s += x;
        st.mean_ms = s / (double)v.size();
    }
    *out = st;
    if (reset) {
        S->lat_ms.clear();
        S->submitted = S->completed = S->rejected = S->batches = S->rows = 0;
        S->peak_bytes = S->bytes_in_use;
    }
    return BMF_OK;
}

}  // extern "C"
