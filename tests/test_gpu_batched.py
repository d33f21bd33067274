"""Batched training: every problem trained inside the batch must
equal the same problem trained alone with the same grid (bit-exact: the
batched launches only regroup independent blocks), and the autotuner must
pick feasible grids."""
import sys

import numpy as np
import pytest

from paper_1907_07410_amd import configs, synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def B():
    from paper_1907_07410_amd import binding
    return binding


def alone(B, m, n, k, b, rat, epochs, lr, reg, order_mode=0):
    G = B.Model(m, n, k, b, order_mode=order_mode)
    G.load_ratings(rat.u, rat.i, rat.r)
    for _ in range(epochs):
        G.epoch(lr, reg)
    return G.get_factors()


def same_bits(a, b):
    return all(np.array_equal(x.view(np.uint32), y.view(np.uint32)) for x, y in zip(a[:4], b[:4]))


@pytest.mark.parametrize("waves", [4, 8])
def test_batch_equals_each_problem_alone(B, waves):
    shapes = [(300, 200, 5000), (1000, 90, 7000), (57, 400, 3000), (800, 800, 0), (2000, 1500, 30000)]
    grids = [4, 8, 2, 16, 2]
    data = [synth.random_coo(m, n, nnz, seed=m + n, dup=True) if nnz else
            synth.Ratings(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
            for m, n, nnz in shapes]
    bt = B.Batch([(m, n) for m, n, _ in shapes], 32, b=grids, waves=waves)
    for p, rat in enumerate(data):
        bt.load(p, rat.u, rat.i, rat.r)
    bt.epochs(3, 0.01, 0.02)
    for p, ((m, n, _), rat) in enumerate(zip(shapes, data)):
        got = bt.problem(p).get_factors()
        want = alone(B, m, n, 32, grids[p], rat, 3, 0.01, 0.02)
        assert same_bits(got, want), p
    ms, launches = bt.timing()
    assert launches == 3 * max(grids) and ms > 0


def test_batch_epochs_in_two_calls_equal_one_call(B):
    shapes = [(400, 300, 6000), (150, 700, 5000)]
    data = [synth.random_coo(m, n, nnz, seed=nnz) for m, n, nnz in shapes]
    outs = []
    for split in ([4], [1, 3]):
        bt = B.Batch([(m, n) for m, n, _ in shapes], 16, b=[4, 8], order_mode=1)
        for p, rat in enumerate(data):
            bt.load(p, rat.u, rat.i, rat.r)
        for e in split:
            bt.epochs(e, 0.01, 0.02)
        outs.append([bt.problem(p).get_factors() for p in range(2)])
    for a, b in zip(*outs):
        assert same_bits(a, b)


def test_batch_autotuned_c4_shape(B, orc):
    """64 problems shaped like the batched workload (uneven sizes, Zipf
    degrees, k=32), scaled down; grids chosen by the autotuner."""
    cfg = configs.BATCHED
    probs = cfg.generate(seed=1, scale=0.06)
    shapes = [(p.m, p.n) for p in probs]
    log("batched: total ratings", sum(len(p.train) for p in probs))
    bt = B.Batch(shapes, cfg.k)
    for q, p in enumerate(probs):
        bt.load(q, p.train.u, p.train.i, p.train.r)
    bt.tune()
    grids = [bt.info(q)[0] for q in range(len(probs))]
    waves = bt.info(0)[1]
    log("chosen grids", sorted(set(grids)), "waves", waves)
    assert waves in (4, 8)
    for q, p in enumerate(probs):
        b = grids[q]
        assert b >= 1
        cb = -(-p.n // b)
        assert cb * cfg.k * 4 <= 160 * 1024
    bt.epochs(2, cfg.lr, cfg.reg)
    rng = np.random.default_rng(0)
    for q in rng.choice(len(probs), 4, replace=False):
        p = probs[q]
        want = alone(B, p.m, p.n, cfg.k, grids[q], p.train, 2, cfg.lr, cfg.reg)
        assert same_bits(bt.problem(int(q)).get_factors(), want), q
    # one problem against the FP64 oracle, one epoch further
    q = int(np.argmin([len(p.train) for p in probs]))
    p = probs[q]
    O = orc.Model(p.m, p.n, cfg.k, grids[q], seed=1001)
    O.load(p.train.u, p.train.i, p.train.r)
    O.epoch(cfg.lr, cfg.reg)
    O.epoch(cfg.lr, cfg.reg)
    P, Q, bu, bi, mu = bt.problem(q).get_factors()
    d = max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(), np.abs(bi - O.bi).max())
    log("batched problem", q, "2 epochs max abs diff vs oracle", d)
    assert d <= 1e-4
