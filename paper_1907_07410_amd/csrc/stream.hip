// Out-of-core training.  Section 6 argues that the block count is not
// bounded, only a block's size is (by the memory of the unit that factorises
// it).  Here the ratings stay in pinned host memory: the partition and the
// step plans are made on the host, the stratum work is laid out stratum after
// stratum, and each epoch copies strata into a ring of device buffers on a
// copy stream while earlier strata's kernels run.  The factor tables
// stay on the device.  The kernels and their results are those of the
// resident path (the same partition, plans and launches).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace bmf {

void PinnedBuf::alloc(size_t n) {
    free_();
    if (n == 0) return;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        BMF_FAIL(BMF_E_NOMEM, "pinned host allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
}

void PinnedBuf::free_() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

void OutOfCore::release() {
    if (copy) (void)hipStreamSynchronize(copy);
    for (int q = 0; q < OOC_BUFS; ++q) {
        if (copied[q]) (void)hipEventDestroy(copied[q]);
        if (used[q]) (void)hipEventDestroy(used[q]);
        copied[q] = used[q] = nullptr;
        used_valid[q] = false;
        stage[q].free_();
    }
    if (copy) (void)hipStreamDestroy(copy);
    copy = nullptr;
    data.free_();
    cu.free_();
    ci.free_();
    cr.free_();
    std::vector<int32_t>().swap(perm);
    s_off.clear();
    s_units.clear();
    ring = 0;
    on = false;
}

namespace {

int bits_for(int64_t count) {  // bits to hold values 0..count-1
    int b = 0;
    while (b < 63 && (1ll << b) < count) ++b;
    return b;
}

int host_threads() { return (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency())); }

// Block (u / rb, i / cb), id row * b + column; inside a block (u, i)
// ascending, equal pairs in input order: the partition the device builds.
void host_partition(Partition &P, std::vector<Rec> &recs, std::vector<int32_t> &perm, const int32_t *u,
                    const int32_t *i, const float *r, int64_t nnz, int64_t m, int64_t n, int b) {
    P.nnz = nnz;
    P.rb = (m + b - 1) / b;
    P.cb = (n + b - 1) / b;
    P.ubits = bits_for(P.rb);
    P.ibits = bits_for(P.cb);
    if (P.ubits + P.ibits > 32)
        BMF_FAIL(BMF_E_RANGE, "a block of " + std::to_string(P.rb) + " x " + std::to_string(P.cb) +
                                  " cells needs more than 32 bits of local index; use a larger block grid");
    const int64_t nb = (int64_t)b * b;
    auto block_of = [&](int64_t t) { return (int64_t)(u[t] / P.rb) * b + i[t] / P.cb; };
    std::vector<int64_t> &bp = P.h_block_ptr;
    bp.assign(nb + 1, 0);
    for (int64_t t = 0; t < nnz; ++t) ++bp[block_of(t) + 1];
    for (int64_t x = 0; x < nb; ++x) bp[x + 1] += bp[x];
    perm.resize(nnz);
    {
        std::vector<int64_t> cur(bp.begin(), bp.end() - 1);
        for (int64_t t = 0; t < nnz; ++t) perm[cur[block_of(t)]++] = (int32_t)t;
    }
    recs.resize(nnz);
    std::atomic<int64_t> next{0};
    auto worker = [&] {
        for (;;) {
            const int64_t blk = next.fetch_add(1);
            if (blk >= nb) return;
            int32_t *beg = perm.data() + bp[blk], *end = perm.data() + bp[blk + 1];
            std::stable_sort(beg, end, [&](int32_t a, int32_t c) { return u[a] != u[c] ? u[a] < u[c] : i[a] < i[c]; });
            const int64_t br = blk / b, bc = blk % b;
            for (int32_t *x = beg; x < end; ++x) {
                const uint32_t lu = (uint32_t)(u[*x] - br * P.rb), li = (uint32_t)(i[*x] - bc * P.cb);
                recs[x - perm.data()] = Rec{(lu << P.ibits) | li, r[*x]};
            }
        }
    };
    const int nt = host_threads();
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

}  // namespace

void ooc_load(Model &M, const int32_t *u, const int32_t *i, const float *r, int64_t nnz) {
    if (nnz < 0) BMF_FAIL(BMF_E_INVAL, "nnz < 0");
    if (nnz > 0 && (!u || !i || !r)) BMF_FAIL(BMF_E_INVAL, "null rating array");
    if (nnz >= (int64_t)INT32_MAX) BMF_FAIL(BMF_E_INVAL, "nnz must be below 2^31");
    for (int64_t t = 0; t < nnz; ++t)
        if (u[t] < 0 || u[t] >= M.m || i[t] < 0 || i[t] >= M.n || !std::isfinite(r[t]))
            BMF_FAIL(BMF_E_RANGE, "rating " + std::to_string(t) + " is out of range or not finite (u=" +
                                      std::to_string(u[t]) + ", i=" + std::to_string(i[t]) + ")");
    // FP64 mean in input order
    double mu = 0.0;
    if (M.mu_mode == 0 && nnz > 0) {
        for (int64_t t = 0; t < nnz; ++t) mu += (double)r[t];
        mu /= (double)nnz;
    }
    Partition P;
    std::vector<Rec> recs;
    std::vector<int32_t> perm;
    host_partition(P, recs, perm, u, i, r, nnz, M.m, M.n, M.b);
    const int b = M.b;
    const int64_t nb = (int64_t)b * b;
    // the kernel the epochs will run, and its units per block
    Plan plan;
    std::vector<SlotRec> flat;
    const bool want_plan = M.sgd_kernel == 2 || (M.sgd_kernel == 0 && plan_pays(nnz, b));
    if (want_plan) plan_host(plan, recs.data(), P.h_block_ptr, P.ibits, P.ubits, P.cb, b, M.k, sgd_max_lds(M.device), flat);
    if (M.sgd_kernel == 2 && !plan.ok)
        BMF_FAIL(BMF_E_STATE, "the LDS-staged SGD kernel needs k <= 128 and an item slice that leaves room for "
                              "user slots in LDS; use SGD kernel 1 or a larger b");
    const int variant = plan.ok ? 2 : 1;
    const std::vector<int64_t> &bptr = variant == 2 ? plan.h_blk_step : P.h_block_ptr;
    const size_t unit = variant == 2 ? PLAN_W * sizeof(SlotRec) : sizeof(Rec);
    const unsigned char *src = variant == 2 ? reinterpret_cast<const unsigned char *>(flat.data())
                                            : reinterpret_cast<const unsigned char *>(recs.data());
    OutOfCore X;
    X.variant = variant;
    X.unit = unit;
    // stratum s: its blocks' units in position order, then its table
    const size_t tbytes = (size_t)(b + 1) * sizeof(int64_t);
    X.s_off.assign(b + 1, 0);
    X.s_units.assign(b, 0);
    size_t max_bytes = 0;
    for (int s = 0; s < b; ++s) {
        int64_t units = 0;
        for (int j = 0; j < b; ++j) {
            const int64_t blk = (int64_t)((j + s) % b) * b + j;
            units += bptr[blk + 1] - bptr[blk];
        }
        X.s_units[s] = units;
        // strata start 256-byte aligned, so that consecutive ones can be
        // copied into one ring buffer with a single copy
        const size_t bytes = ((size_t)units * unit + tbytes + 255) & ~size_t(255);
        X.s_off[s + 1] = X.s_off[s] + (int64_t)bytes;
        max_bytes = std::max(max_bytes, bytes);
    }
    // strata per ring buffer: up to OOC_GROUP of them in OOC_SLOT_BYTES, so
    // that an epoch has b / group copy-to-kernel and kernel-to-copy waits
    // between the streams instead of b of each
    X.group = (int)std::max<size_t>(1, std::min<size_t>(std::min(OOC_GROUP, b), OOC_SLOT_BYTES / std::max<size_t>(1, max_bytes)));
    X.data.alloc((size_t)X.s_off[b]);
    for (int s = 0; s < b; ++s) {
        unsigned char *base = X.data.as<unsigned char>() + X.s_off[s];
        int64_t *tab = reinterpret_cast<int64_t *>(base + (size_t)X.s_units[s] * unit);
        int64_t off = 0;
        for (int j = 0; j < b; ++j) {
            const int64_t blk = (int64_t)((j + s) % b) * b + j;
            const int64_t cnt = bptr[blk + 1] - bptr[blk];
            tab[j] = off;
            if (cnt) std::memcpy(base + (size_t)off * unit, src + (size_t)bptr[blk] * unit, (size_t)cnt * unit);
            off += cnt;
        }
        tab[b] = off;
    }
    X.cu.alloc((size_t)nnz * 4);
    X.ci.alloc((size_t)nnz * 4);
    X.cr.alloc((size_t)nnz * 4);
    if (nnz) {
        std::memcpy(X.cu.p, u, nnz * 4);
        std::memcpy(X.ci.p, i, nnz * 4);
        std::memcpy(X.cr.p, r, nnz * 4);
    }
    X.perm.swap(perm);
    for (int q = 0; q < OOC_BUFS; ++q) {
        X.stage[q].alloc(max_bytes * X.group);
        BMF_HIP(hipEventCreateWithFlags(&X.copied[q], hipEventDisableTiming));
        BMF_HIP(hipEventCreateWithFlags(&X.used[q], hipEventDisableTiming));
    }
    BMF_HIP(hipStreamCreateWithFlags(&X.copy, hipStreamNonBlocking));
    // commit: no resident ratings, the host partition, the plan's shape
    BMF_HIP(hipStreamSynchronize(M.stream));
    M.ooc.release();
    X.on = true;
    std::swap(M.ooc.on, X.on);
    std::swap(M.ooc.variant, X.variant);
    std::swap(M.ooc.unit, X.unit);
    std::swap(M.ooc.group, X.group);
    M.ooc.s_off.swap(X.s_off);
    M.ooc.s_units.swap(X.s_units);
    M.ooc.data.swap(X.data);
    M.ooc.cu.swap(X.cu);
    M.ooc.ci.swap(X.ci);
    M.ooc.cr.swap(X.cr);
    M.ooc.perm.swap(X.perm);
    for (int q = 0; q < OOC_BUFS; ++q) {
        M.ooc.stage[q].swap(X.stage[q]);
        std::swap(M.ooc.copied[q], X.copied[q]);
        std::swap(M.ooc.used[q], X.used[q]);
    }
    std::swap(M.ooc.copy, X.copy);
    M.cu.free_();
    M.ci.free_();
    M.cr.free_();
    M.part.recs.free_();
    M.part.perm.free_();
    M.part.block_ptr.free_();
    M.part.h_block_ptr.swap(P.h_block_ptr);
    M.part.nnz = nnz;
    M.part.rb = P.rb;
    M.part.cb = P.cb;
    M.part.ibits = P.ibits;
    M.part.ubits = P.ubits;
    plan.steps.free_();
    plan.blk_step.free_();
    plan.built = true;
    M.plan.swap(plan);
    M.mu = mu;
    M.loaded = true;
    M.bf16_valid = false;
}

void ooc_epoch(Model &M, const int32_t *order, const HP &hp, int variant) {
    OutOfCore &X = M.ooc;
    const int b = M.b;
    // groups of 1 and 3 strata start the epoch, so that the copy a kernel
    // waits for at the start of an epoch (when nothing of it was queued
    // before) is one stratum's, and each next copy fits under the kernels
    // queued before it; then groups of X.group
    for (int g0 = 0, g1 = 0, gi = 0; g0 < b; g0 = g1, ++gi) {
        g1 = std::min(b, g0 + std::min(X.group, gi == 0 ? 1 : gi == 1 ? 3 : X.group));
        // the ring runs on across epochs, so an epoch's first copies go to
        // buffers the previous epoch's last kernels do not read
        const int q = (int)(X.ring++ % OOC_BUFS);
        // the buffer is free once the kernels that last read it have
        // finished.  The host waits for that before it queues the copy: with
        // the copies of later groups and epochs queued far ahead behind
        // cross-stream waits, single stratum launches took 1.3-2.4 ms instead
        // of 0.27 (about one epoch in two 1-3 ms slower); queued only when
        // the buffer is free, every epoch runs at the resident pace.
        if (X.used_valid[q]) {
            BMF_HIP(hipEventSynchronize(X.used[q]));
            BMF_HIP(hipStreamWaitEvent(X.copy, X.used[q], 0));
        }
        // the group's strata back to back (each its units and its block table
        // behind them), one copy per run of strata adjacent in host memory
        unsigned char *dst = X.stage[q].as<unsigned char>();
        std::vector<size_t> at(g1 - g0);
        size_t off = 0;
        for (int pos = g0; pos < g1;) {
            int end = pos + 1;
            while (end < g1 && order[end] == order[end - 1] + 1) ++end;
            const int s0 = order[pos], s1 = order[end - 1];
            const size_t len = (size_t)(X.s_off[s1 + 1] - X.s_off[s0]);
            BMF_HIP(hipMemcpyAsync(dst + off, X.data.as<unsigned char>() + X.s_off[s0], len, hipMemcpyHostToDevice,
                                   X.copy));
            for (int x = pos; x < end; ++x) at[x - g0] = off + (size_t)(X.s_off[order[x]] - X.s_off[s0]);
            off += len;
            pos = end;
        }
        BMF_HIP(hipEventRecord(X.copied[q], X.copy));
        BMF_HIP(hipStreamWaitEvent(M.stream, X.copied[q], 0));
        for (int pos = g0; pos < g1; ++pos) {
            const int s = order[pos];
            const unsigned char *st = dst + at[pos - g0];
            launch_stratum(M, s, hp, variant,
                           StratumData{st, reinterpret_cast<const int64_t *>(st + (size_t)X.s_units[s] * X.unit), 0});
        }
        BMF_HIP(hipEventRecord(X.used[q], M.stream));
        X.used_valid[q] = true;
    }
}

double ooc_sq_sum(Model &M, const HP *loss_hp) {
    OutOfCore &X = M.ooc;
    const int64_t nnz = M.part.nnz;
    const int64_t chunk = std::min<int64_t>(nnz, (int64_t)1 << 22);
    if (chunk == 0) return 0.0;
    DevBuf du, di, dr;
    du.alloc((size_t)chunk * 4);
    di.alloc((size_t)chunk * 4);
    dr.alloc((size_t)chunk * 4);
    double s = 0.0;
    for (int64_t t0 = 0; t0 < nnz; t0 += chunk) {
        const int64_t c = std::min(chunk, nnz - t0);
        BMF_HIP(hipMemcpyAsync(du.p, X.cu.as<int32_t>() + t0, c * 4, hipMemcpyHostToDevice, M.stream));
        BMF_HIP(hipMemcpyAsync(di.p, X.ci.as<int32_t>() + t0, c * 4, hipMemcpyHostToDevice, M.stream));
        BMF_HIP(hipMemcpyAsync(dr.p, X.cr.as<float>() + t0, c * 4, hipMemcpyHostToDevice, M.stream));
        s += sq_residual_sum(M, du.as<int32_t>(), di.as<int32_t>(), dr.as<float>(), c, loss_hp, M.red);
    }
    return s;
}

}  // namespace bmf
