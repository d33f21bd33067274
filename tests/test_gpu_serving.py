"""Serving engine: results are the same alone and in a mix, equal the
direct top-K and fold-in calls, admission respects the memory budget, and a
Poisson run completes with latency statistics."""
import sys

import numpy as np
import pytest

from paper_1907_07410_amd import serving, synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def B():
    from paper_1907_07410_amd import binding
    return binding


@pytest.fixture(scope="module")
def model(B):
    m, n, k = 20000, 6000, 128
    P, Q, bu, bi, mu = synth.serving_factors(m, n, k, seed=3)
    G = B.Model(m, n, k, 4)
    G.set_factors(P, Q, bu, bi, mu)
    return G, (P, Q, bu, bi, mu)


def same(a, b):
    return np.array_equal(a["items"], b["items"]) and np.array_equal(a["scores"].view(np.uint32),
                                                                     b["scores"].view(np.uint32))


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_in_mix(B, model, precision):
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G, max_batches=2)
    rng = np.random.default_rng(precision)
    probe_u = rng.integers(0, G.m, 37).astype(np.int32)
    probe_items = rng.choice(G.n, 60, replace=False).astype(np.int32)
    probe_r = rng.integers(1, 6, 60).astype(np.float32)
    a = S.poll(S.submit_topk(probe_u, 100, precision))
    af = S.poll(S.submit_foldin(probe_items, probe_r, 50, precision))
    reqs = serving.make_stream(rng, 40, 0, G.m, G.n, Q, bi, mu)
    ids = []
    for q, r in enumerate(reqs):
        if q == 17:
            pid = S.submit_topk(probe_u, 100, precision)
            fid = S.submit_foldin(probe_items, probe_r, 50, precision)
        if r.kind == "topk":
            ids.append(S.submit_topk(r.users, 100, 1 - precision if q % 3 == 0 else precision))
        else:
            ids.append(S.submit_foldin(r.items, r.ratings, 100, precision))
    b = S.poll(pid)
    bf = S.poll(fid)
    for rid in ids:
        S.poll(rid)
    st = S.stats()
    log("mix stats", {k2: st[k2] for k2 in ("batches", "rows", "completed", "p50_ms", "p99_ms")})
    assert st["batches"] < st["completed"]  # requests shared batches
    assert same(a, b)
    assert same(af, bf) and np.array_equal(af["p"].view(np.uint32), bf["p"].view(np.uint32))
    S.close()


def test_server_matches_direct_calls(B, model):
    G, _ = model
    S = B.Server(G)
    rng = np.random.default_rng(9)
    users = rng.integers(0, G.m, 300).astype(np.int32)
    for precision, direct in ((0, G.topk), (1, G.topk_bf16)):
        r = S.poll(S.submit_topk(users, 100, precision))
        di, ds = direct(users, 100)
        assert np.array_equal(r["items"], di)
        assert np.array_equal(r["scores"].view(np.uint32), ds.view(np.uint32))
    items = rng.choice(G.n, 200, replace=False).astype(np.int32)
    rat = rng.integers(1, 6, 200).astype(np.float32)
    p, bu = G.foldin(items, rat, 10, 0.005, 0.05)
    for precision in (0, 1):  # the fold-in itself is FP32 in both
        r = S.poll(S.submit_foldin(items, rat, 100, precision))
        assert np.array_equal(r["p"].view(np.uint32), p.view(np.uint32)) and r["bu"] == bu
    S.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_foldin_topk_matches_oracle(B, orc, model, precision):
    """A new user folded in through the server and then ranked (Section 2.1's
    folding-in, Eq 3's prediction), against the FP64 oracle:
      * p and bu within 1e-5 of the oracle's fold-in;
      * the scoring of the folded-in row: returned items epsilon-valid and
        scores within eps of the FP64 scores of the GPU's own vector;
      * the whole request: items and scores epsilon-valid against the
        oracle's fold-in followed by the oracle's ranking of that vector,
        with eps widened by what the 1e-5 fold-in tolerance can move a
        score (1e-5 (|q_i|_1 + 1))."""
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G)
    rng = np.random.default_rng(40 + precision)
    K = 100
    Qd, bid = Q.astype(np.float64), bi.astype(np.float64)
    eps_scale = (G.k + 8) * 2.0 ** -23
    widen = 1e-5 * (np.abs(Qd).sum(axis=1).max() + 1.0)
    overlap = []
    for nr in (5, 60, 500):
        items = rng.choice(G.n, nr, replace=False).astype(np.int32)
        rat = rng.integers(1, 6, nr).astype(np.float32)
        res = S.poll(S.submit_foldin(items, rat, K, precision))
        it, sc = res["items"][0], res["scores"][0]
        assert len(set(it.tolist())) == K and np.all(np.diff(sc) <= 0)
        op, obu = orc.foldin(Q, bi, mu, items, rat, 10, 0.005, 0.05)
        assert np.abs(res["p"] - op).max() <= 1e-5 and abs(res["bu"] - obu) <= 1e-5, nr
        # scoring of the GPU's folded-in row
        pg = res["p"].astype(np.float64)
        s64 = mu + res["bu"] + bid + Qd @ pg
        eps = eps_scale * (np.abs(Qd * pg).sum(axis=1) + np.abs(bid) + abs(mu + res["bu"])).max()
        kth = np.sort(s64)[::-1][K - 1]
        assert np.all(s64[it] >= kth - eps), (nr, (s64[it] - kth).min(), eps)
        assert np.all(np.abs(sc - s64[it]) <= eps), (nr, np.abs(sc - s64[it]).max(), eps)
        # against the oracle's fold-in and its ranking of the oracle's vector
        oi, os_ = orc.topk_vec(op, obu, Q, bi, mu, G.n)
        o_score = np.empty(G.n)
        o_score[oi] = os_
        eps_o = eps + widen
        assert np.all(o_score[it] >= os_[K - 1] - eps_o), (nr, (o_score[it] - os_[K - 1]).min(), eps_o)
        assert np.all(np.abs(sc - o_score[it]) <= eps_o), (nr, np.abs(sc - o_score[it]).max(), eps_o)
        overlap.append(len(set(it.tolist()) & set(oi[:K].tolist())) / K)
    log("fold-in top-100 overlap with the oracle, precision", precision, overlap)
    assert min(overlap) >= 0.95
    S.close()


def test_admission_by_memory(B, model):
    G, (P, Q, bu, bi, mu) = model
    budget = 64 << 20
    S = B.Server(G, mem_budget_bytes=budget, max_batches=2)
    with pytest.raises(B.BmfError) as ex:
        S.submit_topk(np.zeros(4000, np.int32), 100, 1)  # larger than one batch partition
    assert ex.value.status == B.BMF_E_NOMEM
    rng = np.random.default_rng(5)
    reqs = serving.make_stream(rng, 60, 0, G.m, G.n, Q, bi, mu, batch_range=(1, 600))
    ids = [S.submit_topk(r.users, 100, 1) if r.kind == "topk" else S.submit_foldin(r.items, r.ratings, 100, 1)
           for r in reqs]
    S.drain()
    for rid in ids:
        assert S.poll(rid, wait=False) is not None
    st = S.stats()
    log("admission stats", st)
    assert st["rejected"] == 1 and st["completed"] == 60
    assert 0 < st["peak_bytes"] <= st["budget_bytes"] <= budget
    S.close()


def test_unbatched_configuration_runs_one_request_per_batch(B, model):
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G, max_batches=1, max_requests_per_batch=1)
    rng = np.random.default_rng(6)
    reqs = serving.make_stream(rng, 20, 0, G.m, G.n, Q, bi, mu, batch_range=(1, 256))
    st = serving.run(S, reqs, K=100, precision=0)
    assert st["batches"] == 20 and st["completed"] == 20
    S.close()


def test_poisson_run_reports_latency(B, model):
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G, max_batches=2)
    rng = np.random.default_rng(7)
    reqs = serving.make_stream(rng, 200, 400.0, G.m, G.n, Q, bi, mu, batch_range=(1, 512))
    st = serving.run(S, reqs, K=100, precision=1)
    log("poisson", {k2: st[k2] for k2 in ("req_per_s", "p50_ms", "p99_ms", "batches", "completed")})
    assert st["completed"] == 200 and 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    S.close()


def test_server_rejects_candidate_counts_beyond_selection_capacity(B, model):
    G, _ = model
    for kc in (-1, 1009, 5000):
        with pytest.raises(B.BmfError) as ex:
            B.Server(G, Kc=kc)
        assert ex.value.status == B.BMF_E_INVAL
    B.Server(G, Kc=1008).close()


def test_drain_waits_for_every_request(B, model):
    """After drain, every submitted request is finished: the scheduler marks
    a slot busy before it lets go of the queue to launch the batch, so a
    drain cannot slip between the queue emptying and the batch starting."""
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G)
    rng = np.random.default_rng(17)
    for rep in range(6):
        reqs = serving.make_stream(rng, 80, 0, G.m, G.n, Q, bi, mu, batch_range=(1, 300))
        ids = [S.submit_topk(r.users, 50, rep % 2) if r.kind == "topk" else
               S.submit_foldin(r.items, r.ratings, 50, rep % 2) for r in reqs]
        S.drain()
        for rid in ids:
            assert S.poll(rid, wait=False) is not None, (rep, rid)
    S.close()


def test_concurrent_clients_get_their_own_results(B, model):
    """Four client threads submit and poll at the same time (polls in
    reverse order, mixed precisions and fold-ins): every result equals the
    direct call for the same request, bit for bit, while the scheduler and
    the completion threads run batches of everyone's requests."""
    import threading
    G, (P, Q, bu, bi, mu) = model
    S = B.Server(G)
    rngs = [np.random.default_rng(100 + t) for t in range(4)]
    streams = [serving.make_stream(rngs[t], 30, 0, G.m, G.n, Q, bi, mu, batch_range=(1, 400)) for t in range(4)]
    results = [None] * 4
    errors = []

    def client(t):
        try:
            ids = []
            for q, r in enumerate(streams[t]):
                prec = (q + t) % 2
                if r.kind == "topk":
                    ids.append((S.submit_topk(r.users, 100, prec), r, prec))
                else:
                    ids.append((S.submit_foldin(r.items, r.ratings, 100, prec), r, prec))
            results[t] = [(S.poll(rid, wait=True), r, prec) for rid, r, prec in reversed(ids)]
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not errors and all(not th.is_alive() for th in threads)
    n = 0
    for t in range(4):
        for res, r, prec in results[t]:
            if r.kind == "topk":
                di, ds = (G.topk_bf16 if prec else G.topk)(r.users, 100)
                assert np.array_equal(res["items"], di)
                assert np.array_equal(res["scores"].view(np.uint32), ds.view(np.uint32))
            else:
                p, b_ = G.foldin(r.items, r.ratings, 10, 0.005, 0.05)
                assert np.array_equal(res["p"].view(np.uint32), p.view(np.uint32)) and res["bu"] == b_
            n += 1
    st = S.stats()
    log("concurrent clients", n, "requests in", st["batches"], "batches")
    assert n == 120 and st["completed"] == 120
    S.close()
