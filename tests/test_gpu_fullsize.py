"""Full-size parity.

Mid-scale workload (138,000 x 27,000, 18M training ratings, k=64, 64 x 64
blocks) in the launch configuration the benchmark times: partition
bit-exact, factors within 1e-4 after one epoch, test RMSE within 1e-3 after
20 epochs.

Large-scale workload (480,000 x 17,800, 90M training ratings, k=128,
128 x 128 blocks): partition bit-exact, factors within 1e-4 after one
epoch, test and training RMSE within 1e-3 after 20 epochs, then top-100 for
20,000 users in FP32 (every answer epsilon-valid against FP64 scores on
sampled users) and in BF16 with FP32 rescoring (recall@100 against FP32 of
at least 0.99).

Serving tables (1,000,000 x 100,000, k = 128): server results equal the
direct BF16 calls, BF16 recall against FP32 of at least 0.99, epsilon-valid
answers on sampled users.  The same tables with a decaying spectrum (factor
f scaled by 1/sqrt(1 + f)): BF16 recall against FP32 of at least 0.99.

Batched workload at 1/4 linear scale (the benchmark runs it at full size and
checks four problems the same way): sampled problems equal the
same problems trained alone, bit for bit; after the configuration's 10
epochs, three problems' training RMSE is within 1e-3 of the oracle's on
the same grids (the batched problems have no held-out split).

The oracle runs its threaded stratum mode (identical results for any thread
count)."""
import os
import sys

import numpy as np
import pytest

from paper_1907_07410_amd import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def mid():
    return configs.MID.generate(1)


def test_mid_scale_parity(orc, mid):
    from paper_1907_07410_amd import binding as B
    cfg = configs.MID
    tr, te = mid.train, mid.test
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    log("mid-scale: loading", len(tr), "ratings; oracle threads", threads)
    G = B.Model(mid.m, mid.n, cfg.k, cfg.b, seed=1001, order_mode=0)
    G.load_ratings(tr.u, tr.i, tr.r)
    O = orc.Model(mid.m, mid.n, cfg.k, cfg.b, seed=1001, order_mode=0)
    O.load(tr.u, tr.i, tr.r)
    bp, perm = G.get_partition(len(tr))
    assert np.array_equal(bp, O.block_ptr) and np.array_equal(perm, O.perm)
    log("partition bit-exact")
    G.epoch(cfg.lr, cfg.reg)
    O.epoch(cfg.lr, cfg.reg, threads=threads)
    P, Q, bu, bi, mu = G.get_factors()
    d = max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(), np.abs(bi - O.bi).max())
    log("one epoch max abs diff", d)
    assert d <= 1e-4
    for e in range(1, cfg.epochs):
        G.epoch(cfg.lr, cfg.reg)
        O.epoch(cfg.lr, cfg.reg, threads=threads)
    rg, ro = G.rmse(te.u, te.i, te.r), O.rmse(te.u, te.i, te.r)
    log("20 epochs test rmse gpu", rg, "oracle", ro)
    assert abs(rg - ro) <= 1e-3
    tg, to = G.rmse(), O.rmse()
    log("20 epochs train rmse gpu", tg, "oracle", to)
    assert abs(tg - to) <= 1e-3


def test_large_scale_parity_and_bf16_scoring(orc):
    from paper_1907_07410_amd import binding as B
    from test_gpu_parity import eps_valid
    cfg = configs.LARGE
    large = cfg.generate(1)
    tr = large.train
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    log("large-scale: loading", len(tr), "ratings")
    G = B.Model(large.m, large.n, cfg.k, cfg.b, seed=1001, order_mode=0)
    G.load_ratings(tr.u, tr.i, tr.r)
    O = orc.Model(large.m, large.n, cfg.k, cfg.b, seed=1001, order_mode=0)
    O.load(tr.u, tr.i, tr.r)
    bp, perm = G.get_partition(len(tr))
    assert np.array_equal(bp, O.block_ptr) and np.array_equal(perm, O.perm)
    log("partition bit-exact")
    G.epoch(cfg.lr, cfg.reg)
    O.epoch(cfg.lr, cfg.reg, threads=threads)
    P, Q, bu, bi, mu = G.get_factors()
    d = max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(), np.abs(bi - O.bi).max())
    log("one epoch max abs diff", d)
    assert d <= 1e-4
    for e in range(1, cfg.epochs):
        G.epoch(cfg.lr, cfg.reg)
        O.epoch(cfg.lr, cfg.reg, threads=threads)
    te = large.test
    rg, ro = G.rmse(te.u, te.i, te.r), O.rmse(te.u, te.i, te.r)
    log(cfg.epochs, "epochs test rmse gpu", rg, "oracle", ro)
    assert abs(rg - ro) <= 1e-3
    tg, to = G.rmse(), O.rmse()
    log(cfg.epochs, "epochs train rmse gpu", tg, "oracle", to)
    assert abs(tg - to) <= 1e-3
    P, Q, bu, bi, mu = G.get_factors()
    del O
    rng = np.random.default_rng(3)
    users = rng.choice(large.m, 20000, replace=False).astype(np.int32)
    K = 100
    fi, fs = G.topk(users, K)
    bi_, bs = G.topk_bf16(users, K)
    recall = float(np.mean([len(set(a) & set(b)) / K for a, b in zip(fi, bi_)]))
    log("large-scale bf16 recall@100 vs fp32 over", len(users), "users:", recall)
    assert recall >= 0.99
    pick = rng.choice(len(users), 24, replace=False)
    eps_valid(fi[pick], fs[pick], P, Q, bu, bi, mu, users[pick], K, (cfg.k + 8) * 2.0 ** -23)
    eps_valid(bi_[pick], bs[pick], P, Q, bu, bi, mu, users[pick], K, (cfg.k + 8) * 2.0 ** -23)


def test_serving_tables_full_size():
    """The serving workload's tables (1,000,000 x 100,000, k = 128): through
    the server with its default configuration, a mixed stream's top-100
    results equal the direct BF16 calls bit for bit, BF16 recall against FP32
    is at least 0.99, and sampled users' answers are epsilon-valid against
    FP64 scores."""
    from paper_1907_07410_amd import binding as B, serving, synth
    from test_gpu_parity import eps_valid
    sc = configs.SERVING
    P, Q, bu, bi, mu = synth.serving_factors(sc.m, sc.n, sc.k, seed=5)
    G = B.Model(sc.m, sc.n, sc.k, 1)
    G.set_factors(P, Q, bu, bi, mu)
    rng = np.random.default_rng(21)
    reqs = [r for r in serving.make_stream(rng, 40, 0, sc.m, sc.n, Q, bi, mu, topk_frac=1.0,
                                           batch_range=(1, 2048))]
    S = B.Server(G, mem_budget_bytes=2 << 30)
    ids = [S.submit_topk(r.users, sc.K, 1) for r in reqs]
    S.drain()
    users_all, items_srv = [], []
    for r, rid in zip(reqs, ids):
        res = S.poll(rid, wait=True)
        di, ds = G.topk_bf16(r.users, sc.K)
        assert np.array_equal(res["items"], di) and np.array_equal(res["scores"].view(np.uint32), ds.view(np.uint32))
        users_all.append(r.users)
        items_srv.append(di)
    S.close()
    users = np.concatenate(users_all)
    bf = np.concatenate(items_srv)
    fi, fs = G.topk(users, sc.K)
    recall = float(np.mean([len(set(a) & set(b)) / sc.K for a, b in zip(fi, bf)]))
    log("serving tables: bf16 recall@100 vs fp32 over", len(users), "users:", recall)
    assert recall >= 0.99
    pick = rng.choice(len(users), 16, replace=False)
    bs = np.concatenate([G.topk_bf16(users[pick], sc.K)[1]])
    eps_valid(bf[pick], bs, P, Q, bu, bi, mu, users[pick], sc.K, (sc.k + 8) * 2.0 ** -23)
    eps_valid(fi[pick], fs[pick], P, Q, bu, bi, mu, users[pick], sc.K, (sc.k + 8) * 2.0 ** -23)


def test_serving_tables_decaying_spectrum():
    """Serving-size tables (1,000,000 x 100,000, k = 128) whose factor f is
    scaled by 1/sqrt(1 + f), the case with more near ties: BF16 recall@100
    against FP32 is at least 0.99 over 4096 users; sampled FP32 answers are
    epsilon-valid against FP64 scores, and the BF16 path's rescored scores
    are within the same epsilon of the FP64 scores of the items it returns."""
    from paper_1907_07410_amd import binding as B, synth
    from test_gpu_parity import eps_valid
    sc = configs.SERVING
    P, Q, bu, bi, mu = synth.serving_factors(sc.m, sc.n, sc.k, seed=6, correlated=True)
    G = B.Model(sc.m, sc.n, sc.k, 1)
    G.set_factors(P, Q, bu, bi, mu)
    rng = np.random.default_rng(22)
    users = rng.integers(0, sc.m, 4096).astype(np.int32)
    fi, fs = G.topk(users, sc.K)
    bi_, bs = G.topk_bf16(users, sc.K)
    recall = float(np.mean([len(set(a) & set(b)) / sc.K for a, b in zip(fi, bi_)]))
    log("decaying-spectrum tables: bf16 recall@100 vs fp32 over", len(users), "users:", recall)
    assert recall >= 0.99
    pick = rng.choice(len(users), 16, replace=False)
    eps_scale = (sc.k + 8) * 2.0 ** -23
    eps_valid(fi[pick], fs[pick], P, Q, bu, bi, mu, users[pick], sc.K, eps_scale)
    Qd = Q.astype(np.float64)
    for row in pick:
        u = users[row]
        s64 = mu + float(bu[u]) + bi.astype(np.float64) + Qd @ P[u].astype(np.float64)
        eps = eps_scale * (np.abs(Qd * P[u].astype(np.float64)).sum(axis=1) + np.abs(bi) + abs(mu + bu[u])).max()
        it = bi_[row]
        assert len(set(it.tolist())) == sc.K and np.all(np.diff(bs[row]) <= 0)
        assert np.all(np.abs(bs[row] - s64[it]) <= eps)
    G.close()


def test_batched_quarter_scale_equals_alone(orc):
    """The batched workload at 1/4 linear scale (64 problems, users and
    items at 1/4): after two batched epochs with autotuned grids, eight of
    the problems equal the same problems trained alone on the same grids,
    bit for bit.  After the configuration's 10 epochs the smallest, the
    largest and a middle problem have a training RMSE within 1e-3 of the
    FP64 oracle trained on the same grid."""
    from paper_1907_07410_amd import binding as B
    bc = configs.BATCHED
    probs = bc.generate(1, 0.25, workers=min(16, os.cpu_count() or 1))
    bt = B.Batch([(p.m, p.n) for p in probs], bc.k, seed=1001)
    for q, p in enumerate(probs):
        bt.load(q, p.train.u, p.train.i, p.train.r)
    bt.tune()
    bt.epochs(2, bc.lr, bc.reg)
    for q in range(0, 64, 8):
        p = probs[q]
        b = bt.info(q)[0]
        G = B.Model(p.m, p.n, bc.k, b, seed=1001)
        G.load_ratings(p.train.u, p.train.i, p.train.r)
        for _ in range(2):
            G.epoch(bc.lr, bc.reg)
        got, want = bt.problem(q).get_factors(), G.get_factors()
        for x, y in zip(got[:4], want[:4]):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), q
        log("batched problem", q, "grid", b, "ratings", len(p.train), "bit-identical")
    bt.epochs(bc.epochs - 2, bc.lr, bc.reg)
    sizes = [len(p.train) for p in probs]
    order = np.argsort(sizes)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    for q in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        p = probs[q]
        b = bt.info(q)[0]
        O = orc.Model(p.m, p.n, bc.k, b, seed=1001, order_mode=0)
        O.load(p.train.u, p.train.i, p.train.r)
        for _ in range(bc.epochs):
            O.epoch(bc.lr, bc.reg, threads=threads)
        tg, to = bt.problem(q).rmse(), O.rmse()
        log("batched problem", q, "grid", b, "ratings", len(p.train), bc.epochs, "epochs train rmse gpu", tg,
            "oracle", to)
        assert abs(tg - to) <= 1e-3
    bt.close()
