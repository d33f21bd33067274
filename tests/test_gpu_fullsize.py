"""Full-size parity on the mid-scale workload (138,000 x 27,000, 18M
training ratings, k=64, 64 x 64 blocks) in the launch configuration the
benchmark times: partition bit-exact, factors within 1e-4 after one epoch,
test RMSE within 1e-3 after 20 epochs.  The oracle runs its threaded stratum
mode (identical results for any thread count)."""
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
