"""Host-side logic outside the library, on the CPU: the synthetic workload
generators (shapes, splits, value ranges, degree caps) and the benchmark's
algorithmic-byte and critical-path counts (checked against brute force on
small cases)."""
import numpy as np
import pytest

import bench
from paper_1907_07410_amd import configs, synth


def test_capped_zipf_degrees_sum_and_cap():
    for count, total, s, cap in ((100, 3000, 1.1, 50), (6040, 1_000_209, 0.35, 3883), (10, 100, 2.0, 10)):
        d = synth.capped_zipf_degrees(count, total, s, cap)
        assert d.sum() == total and d.max() <= cap and d.min() >= 0
        assert np.all(np.diff(d) <= 0)  # rank order: non-increasing
    with pytest.raises(ValueError):
        synth.capped_zipf_degrees(10, 101, 1.0, 10)


def test_paper_workload_shape():
    c = configs.PAPER_ML1M
    p = c.generate(1, scale=0.1)
    assert (p.m, p.n) == (604, 388)
    total = len(p.train) + len(p.test)
    assert total == round(c.nnz * 0.1)
    assert len(p.train) == round(0.8 * total)
    allk = np.concatenate([p.train.u.astype(np.int64) * p.n + p.train.i, p.test.u.astype(np.int64) * p.n + p.test.i])
    assert np.unique(allk).shape[0] == total  # distinct (u, i) pairs
    r = np.concatenate([p.train.r, p.test.r])
    assert set(np.unique(r)) <= {1.0, 2.0, 3.0, 4.0, 5.0}


def test_mid_workload_half_stars_small_scale():
    p = configs.MID.generate(1, scale=0.02)
    r = p.train.r
    assert r.min() >= 0.5 and r.max() <= 5.0 and np.all(np.round(r * 2) == r * 2)


def test_batched_generation_same_with_threads():
    bc = configs.BATCHED
    one = bc.generate(3, scale=0.02)
    many = bc.generate(3, scale=0.02, workers=4)
    assert len(one) == len(many) == bc.nprob
    for a, c in zip(one, many):
        assert (a.m, a.n) == (c.m, c.n)
        assert np.array_equal(a.train.u, c.train.u) and np.array_equal(a.train.i, c.train.i)
        assert np.array_equal(a.train.r, c.train.r)


@pytest.mark.parametrize("rounding", ["int", "half"])
def test_pair_and_value_draws_do_not_depend_on_threads(rounding):
    """The chunked draws take one child stream per chunk, so the thread
    count changes nothing; pairs are distinct and degrees follow the caps."""
    out = []
    for w in (1, 3):
        rng = np.random.default_rng(11)
        u, i = synth.sample_pairs_zipf(5000, 700, 300000, 1.0, 1.1, rng, workers=w)
        r = synth.planted_values(u, i, 5000, 700, 4, 0.3, 0.5, 3.5, rounding, rng, chunk=40000, workers=w)
        out.append((u, i, r))
    for a, c in zip(out[0], out[1]):
        assert np.array_equal(a, c)
    u, i, r = out[0]
    k = u.astype(np.int64) * 700 + i
    assert np.unique(k).size == k.size == 300000
    assert np.bincount(u, minlength=5000).max() <= 700 and np.bincount(i, minlength=700).max() <= 5000
    lo = 1.0 if rounding == "int" else 0.5
    assert r.min() >= lo and r.max() <= 5.0


def brute(u, i, m, n, b, k):
    rb, cb = -(-m // b), -(-n // b)
    users, items = set(), set()
    cnt = {}
    for uu, ii in zip(u.tolist(), i.tolist()):
        blk = (uu // rb, ii // cb)
        users.add((blk, uu))
        items.add((blk, ii))
        cnt[blk] = cnt.get(blk, 0) + 1
    algo = len(u) * 8 + (len(users) + len(items)) * (k + 1) * 4 * 2
    crit = sum(max(cnt.get(((j + s) % b, j), 0) for j in range(b)) for s in range(b))
    return algo, len(users), len(items), crit


@pytest.mark.parametrize("m,n,b,nnz", [(50, 40, 4, 600), (37, 91, 5, 900), (10, 10, 3, 30)])
def test_algorithmic_bytes_and_critical_path(m, n, b, nnz):
    rat = synth.random_coo(m, n, nnz, seed=m + b)
    k = 16
    algo, nu, ni = bench.algorithmic_bytes(rat.u, rat.i, m, n, b, k)
    cp, mx, mean = bench.critical_path(rat.u, rat.i, m, n, b)
    ba, bu, bi, bc = brute(rat.u, rat.i, m, n, b, k)
    assert (algo, nu, ni, cp) == (ba, bu, bi, bc)
    assert mean == pytest.approx(nnz / (b * b))
