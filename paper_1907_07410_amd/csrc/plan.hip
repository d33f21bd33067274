// Execution plan of the LDS-staged SGD kernel: a list schedule of each
// block's ratings.
//
// Algorithm 2 visits a block's ratings row by row (users ascending, items
// ascending within a user).  The update of Eqs 10-13 for rating (u, i)
// reads and writes only p_u, bu_u, q_i and bi_i, so two ratings that share
// neither the user nor the item commute exactly; any order in which every
// user's ratings and every item's ratings keep their row-major order gives
// bit-identical results.  The plan packs the ratings into steps of W = 4
// mutually independent ratings (one per 16-lane group of the kernel's chain
// wavefront) by list scheduling: each step takes the lowest-indexed ratings
// whose user and item predecessors ran in earlier steps.
//
// User rows live in LDS slots while a user is active in the block.  The
// kernel's helper wavefronts load a user's row into its slot during the
// chunk (CH steps) before the user's first step and write it back during
// the chunk after its last step, so a slot freed in chunk a is handed out
// again only to a user whose first step is in chunk a + 3 or later.  New
// users may start out of order (a later user whose first rating is ready
// takes a free slot while a lower user still waits for an item
// predecessor).  That cannot stall the plan: the lowest active user always
// has a runnable rating, and the lowest unstarted user becomes ready when
// the users before it finish, at the latest one step after the last of them
// frees its slot, which becomes usable two chunks later and goes to the
// lowest ready user.  The loop still checks for a stall and then plans the
// block again with users starting in order.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <deque>
#include <mutex>
#include <queue>
#include <thread>

#include "internal.h"

namespace bmf {

namespace {

using HeapItem = std::pair<int32_t, int32_t>;  // (key, rating)
using MinHeap = std::priority_queue<HeapItem, std::vector<HeapItem>, std::greater<HeapItem>>;

struct Scratch {
    std::vector<int32_t> next_u, next_i, npred, earliest, slot, last_item;
    std::vector<uint8_t> first, started;
};

// One attempt; returns false on a stall (only possible when users start
// out of order).
bool schedule_block(const uint32_t *ui, int64_t n, int ibits, int cb, int S, int CH, bool in_order,
                    std::vector<PlanEntry> &out, Scratch &z) {
    const uint32_t imask = (1u << ibits) - 1u;
    const int N = (int)n;
    z.next_u.assign(N, -1);
    z.next_i.assign(N, -1);
    z.npred.assign(N, 0);
    z.earliest.assign(N, 0);
    z.slot.assign(N, -1);
    z.first.assign(N, 0);
    z.started.assign(N, 0);
    if ((int)z.last_item.size() < cb) z.last_item.resize(cb);
    for (int x = 0; x < N; ++x) z.last_item[ui[x] & imask] = -1;
    for (int x = 0; x < N; ++x) {
        const uint32_t u = ui[x] >> ibits, it = ui[x] & imask;
        z.first[x] = (x == 0 || (ui[x - 1] >> ibits) != u);
        if (!z.first[x]) {
            z.next_u[x - 1] = x;
            z.npred[x]++;
        }
        const int li = z.last_item[it];
        if (li >= 0) {
            z.next_i[li] = x;
            z.npred[x]++;
        }
        z.last_item[it] = x;
    }
    MinHeap pend, ready_cont, ready_new;
    for (int x = 0; x < N; ++x)
        if (z.npred[x] == 0) pend.push({0, x});
    std::deque<std::pair<int32_t, int32_t>> free_slots;  // (slot, first chunk it may be loaded for)
    for (int q = 0; q < S; ++q) free_slots.push_back({q, 0});
    int next_new = 0;  // first rating of the lowest unstarted user
    out.clear();
    int done = 0;
    for (int64_t s = 0; done < N; ++s) {
        const int chunk = (int)(s / CH);
        while (!pend.empty() && pend.top().first <= s) {
            const int x = pend.top().second;
            pend.pop();
            (z.first[x] ? ready_new : ready_cont).push({x, x});
        }
        int picked = 0;
        while (picked < PLAN_W) {
            const int cc = ready_cont.empty() ? -1 : ready_cont.top().second;
            int cn = -1;
            if (!ready_new.empty() && !free_slots.empty() && free_slots.front().second <= chunk) {
                cn = ready_new.top().second;
                if (in_order && cn != next_new) cn = -1;
            }
            int x;
            if (cc >= 0 && (cn < 0 || cc < cn)) {
                x = cc;
                ready_cont.pop();
            } else if (cn >= 0) {
                x = cn;
                ready_new.pop();
            } else {
                break;
            }
            if (z.first[x]) {
                z.slot[x] = free_slots.front().first;
                free_slots.pop_front();
                z.started[x] = 1;
                if (x == next_new) {
                    int y = x + 1;
                    while (y < N && (!z.first[y] || z.started[y])) ++y;
                    next_new = y;
                }
            } else {
                z.slot[x] = z.slot[x - 1];
            }
            if (z.next_u[x] < 0) free_slots.push_back({z.slot[x], chunk + 3});
            out.push_back(PlanEntry{x, z.slot[x]});
            ++done;
            ++picked;
            for (const int y : {z.next_u[x], z.next_i[x]}) {
                if (y < 0) continue;
                z.earliest[y] = std::max<int32_t>(z.earliest[y], (int32_t)s + 1);
                if (--z.npred[y] == 0) pend.push({z.earliest[y], y});
            }
        }
        for (; picked < PLAN_W; ++picked) out.push_back(PlanEntry{-1, S});
        // Nothing can run now and nothing ever will: every slot is held and
        // no held user has a rating in flight.
        if (done < N && pend.empty() && ready_cont.empty() && free_slots.empty()) return false;
    }
    return true;
}

}  // namespace

int plan_kp(int k) {
    for (int F = 1; F <= 8; F *= 2)
        if (16 * F >= k) return 16 * F;
    return 0;
}

int64_t plan_block(const uint32_t *ui, int64_t n, int ibits, int cb, int S, int CH, std::vector<PlanEntry> &out) {
    if (S < 1 || CH < 1 || S > PLAN_MAX_SLOTS) BMF_FAIL(BMF_E_INVAL, "plan needs 1 to 4095 user slots and CH >= 1");
    if (n >= INT32_MAX) BMF_FAIL(BMF_E_RANGE, "block too large to plan");
    Scratch z;
    if (!schedule_block(ui, n, ibits, cb, S, CH, false, out, z)) {
        const bool ok = schedule_block(ui, n, ibits, cb, S, CH, true, out, z);
        if (!ok) BMF_FAIL(BMF_E_STATE, "block plan stalled with users starting in order");
    }
    return (int64_t)out.size() / PLAN_W;
}

int64_t chain_depth(const int32_t *u, const int32_t *i, int64_t n) {
    if (n <= 0) return 0;
    const int32_t umax = *std::max_element(u, u + n), imax = *std::max_element(i, i + n);
    std::vector<int64_t> du((size_t)umax + 1, 0), di((size_t)imax + 1, 0);
    int64_t best = 0;
    for (int64_t x = 0; x < n; ++x) {
        // one after the last rating of its user and the last of its item
        const int64_t d = std::max(du[u[x]], di[i[x]]) + 1;
        du[u[x]] = di[i[x]] = d;
        best = std::max(best, d);
    }
    return best;
}

int plan_slots(int kp, int64_t cb, int CH, int max_lds) {
    max_lds = std::min(max_lds, PLAN_LDS_BYTES);
    const PlanLds L0 = plan_lds(kp, cb, 0, CH);
    const int64_t room = (int64_t)max_lds - (int64_t)L0.total;
    if (room <= 0) return 0;
    int64_t S = room / (kp * 4 + 4) - 1;
    while (S > 0 && (int64_t)plan_lds(kp, cb, (int)S, CH).total > max_lds) --S;
    return (int)std::min<int64_t>(S, PLAN_MAX_SLOTS);
}

bool plan_host(Plan &out, const Rec *recs, const std::vector<int64_t> &block_ptr, int ibits, int ubits, int64_t cb,
               int b, int k, int max_lds, std::vector<SlotRec> &flat) {
    out.ok = false;
    out.built = true;
    flat.clear();
    const int kp = plan_kp(k);
    if (!kp || cb + 1 > (1 << 16) || ubits > 30) return false;
    const int CH = PLAN_CH;
    const int S = plan_slots(kp, cb, CH, max_lds);
    if (S < PLAN_MIN_SLOTS) return false;
    const PlanLds L = plan_lds(kp, cb, S, CH);
    const int64_t nblk = (int64_t)b * b;
    const uint32_t imask = (1u << ibits) - 1u;
    std::vector<std::vector<SlotRec>> per(nblk);
    std::atomic<int64_t> next{0};
    std::atomic<bool> failed{false};
    std::string fail_msg;
    std::mutex fail_mu;
    auto worker = [&] {
        std::vector<uint32_t> ui;
        std::vector<PlanEntry> ent;
        for (;;) {
            const int64_t blk = next.fetch_add(1);
            if (blk >= nblk || failed.load()) return;
            const int64_t beg = block_ptr[blk], end = block_ptr[blk + 1];
            const int64_t cnt = end - beg;
            ui.resize(cnt);
            for (int64_t x = 0; x < cnt; ++x) ui[x] = recs[beg + x].ui;
            try {
                plan_block(ui.data(), cnt, ibits, (int)cb, S, CH, ent);
            } catch (const Error &e) {
                std::lock_guard<std::mutex> g(fail_mu);
                fail_msg = e.msg;
                failed = true;
                return;
            }
            auto &o = per[blk];
            o.resize(ent.size());
            for (size_t q = 0; q < ent.size(); ++q) {
                const int x = ent[q].x;
                if (x < 0) {
                    o[q] = SlotRec{(uint32_t)(L.q + (size_t)cb * L.row_bytes), 0.f,
                                   (uint32_t)(L.u + (size_t)S * L.row_bytes), 0u};
                    continue;
                }
                const uint32_t u = ui[x] >> ibits;
                const bool first = x == 0 || (ui[x - 1] >> ibits) != u;
                const bool last = x + 1 == cnt || (ui[x + 1] >> ibits) != u;
                o[q] = SlotRec{(uint32_t)(L.q + (size_t)(ui[x] & imask) * L.row_bytes), recs[beg + x].r,
                               (uint32_t)(L.u + (size_t)ent[q].slot * L.row_bytes),
                               u | (first ? PLAN_FIRST : 0u) | (last ? PLAN_LAST : 0u)};
            }
        }
    };
    const int nt = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
    if (failed) BMF_FAIL(BMF_E_STATE, fail_msg);
    out.h_blk_step.assign(nblk + 1, 0);
    for (int64_t blk = 0; blk < nblk; ++blk)
        out.h_blk_step[blk + 1] = out.h_blk_step[blk] + (int64_t)per[blk].size() / PLAN_W;
    out.total_steps = out.h_blk_step[nblk];
    flat.reserve(out.total_steps * PLAN_W);
    for (auto &v : per) {
        flat.insert(flat.end(), v.begin(), v.end());
        std::vector<SlotRec>().swap(v);
    }
    out.kp = kp;
    out.S = S;
    out.CH = CH;
    out.ok = true;
    return true;
}

void build_plan(Plan &out, const Partition &part, int b, int k, int max_lds, hipStream_t s) {
    std::vector<Rec> recs(part.nnz);
    if (part.nnz) {
        BMF_HIP(hipMemcpyAsync(recs.data(), part.recs.p, part.nnz * sizeof(Rec), hipMemcpyDeviceToHost, s));
        BMF_HIP(hipStreamSynchronize(s));
    }
    std::vector<SlotRec> flat;
    if (!plan_host(out, recs.data(), part.h_block_ptr, part.ibits, part.ubits, part.cb, b, k, max_lds, flat)) return;
    out.ok = false;
    const int64_t nblk = (int64_t)b * b;
    out.steps.alloc(std::max<size_t>(16, flat.size() * sizeof(SlotRec)));
    out.blk_step.alloc((nblk + 1) * sizeof(int64_t));
    if (!flat.empty())
        BMF_HIP(hipMemcpyAsync(out.steps.p, flat.data(), flat.size() * sizeof(SlotRec), hipMemcpyHostToDevice, s));
    BMF_HIP(hipMemcpyAsync(out.blk_step.p, out.h_blk_step.data(), (nblk + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    BMF_HIP(hipStreamSynchronize(s));
    out.ok = true;
}

}  // namespace bmf
