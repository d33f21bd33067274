"""Pins of the oracle's incremental path (Section 6): new ratings become new
blocks factorised on their own, then every rating trains together.

* growth keeps learned rows and gives new rows exactly the initial values of
  a model created at the new size;
* during the new-ratings phase, a row no new rating touches stays
  bit-identical (new users x new items leaves every old row alone; new users
  x old items leaves old users alone);
* the union becomes the training set: its partition is the partition of the
  concatenated ratings on the grown grid;
* with no new ratings and no growth the model is unchanged;
* quality: on a planted data set cut into an old part and new users and
  items, the incremental model ends within 0.01 test RMSE of training from
  scratch on everything for the same number of passes over the union."""
import numpy as np
import pytest

from paper_1907_07410_amd import synth

HP = (0.01, 0.02) * 4


def planted(seed=5, m=1200, n=600, nnz=60000):
    rng = np.random.default_rng(seed)
    u, i = synth.sample_pairs_zipf(m, n, nnz, 0.6, 0.6, rng)
    r = synth.planted_values(u, i, m, n, 8, 0.4, 0.5, 3.5, "none", rng)
    return synth.split(synth.Ratings(u, i, r), 0.9, rng)


def snapshot(O):
    return O.P.copy(), O.Q.copy(), O.bu.copy(), O.bi.copy()


def test_growth_keeps_rows_and_seeds_new_ones(orc):
    tr, _ = planted()
    m0, n0 = 1000, 500
    keep = (tr.u < m0) & (tr.i < n0)
    O = orc.Model(m0, n0, 8, 4, seed=77)
    O.load(tr.u[keep], tr.i[keep], tr.r[keep])
    for _ in range(3):
        O.epoch(hp=HP)
    P, Q, bu, bi = snapshot(O)
    O.add_ratings(1200, 600, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), HP, 2)
    F = orc.Model(1200, 600, 8, 4, seed=77)
    assert np.array_equal(O.P[:m0], P) and np.array_equal(O.Q[:n0], Q)
    assert np.array_equal(O.bu[:m0], bu) and np.array_equal(O.bi[:n0], bi)
    assert np.array_equal(O.P[m0:], F.P[m0:]) and np.array_equal(O.Q[n0:], F.Q[n0:])
    assert not O.bu[m0:].any() and not O.bi[n0:].any()
    assert not np.array_equal(P, F.P[:m0])  # the kept rows were trained


@pytest.mark.parametrize("new_items", [True, False])
def test_untouched_rows_stay_during_new_phase(orc, new_items):
    tr, _ = planted()
    m0, n0 = 1000, 500
    old = (tr.u < m0) & (tr.i < n0)
    new = (tr.u >= m0) & ((tr.i >= n0) if new_items else (tr.i < n0))
    assert new.sum() > 100
    O = orc.Model(m0, n0, 8, 4, seed=77)
    O.load(tr.u[old], tr.i[old], tr.r[old])
    for _ in range(3):
        O.epoch(hp=HP)
    P, Q, bu, bi = snapshot(O)
    O.add_ratings(1200, 600, tr.u[new], tr.i[new], tr.r[new], HP, 2)
    assert np.array_equal(O.P[:m0], P) and np.array_equal(O.bu[:m0], bu)
    if new_items:
        assert np.array_equal(O.Q[:n0], Q) and np.array_equal(O.bi[:n0], bi)
    else:
        assert not np.array_equal(O.Q[:n0], Q)
    F = orc.Model(1200, 600, 8, 4, seed=77)
    assert not np.array_equal(O.P[m0:], F.P[m0:])  # the new users were trained


def test_union_becomes_training_set(orc):
    tr, _ = planted()
    m0, n0 = 1000, 500
    old = (tr.u < m0) & (tr.i < n0)
    O = orc.Model(m0, n0, 8, 4, seed=77)
    O.load(tr.u[old], tr.i[old], tr.r[old])
    O.add_ratings(1200, 600, tr.u[~old], tr.i[~old], tr.r[~old], HP, 1)
    au = np.concatenate([tr.u[old], tr.u[~old]])
    ai = np.concatenate([tr.i[old], tr.i[~old]])
    bp, perm = orc.partition(1200, 600, 4, au, ai)
    assert np.array_equal(O.block_ptr, bp) and np.array_equal(O.perm, perm)
    assert O.mu == pytest.approx(float(np.concatenate([tr.r[old], tr.r[~old]]).astype(np.float64).mean()), abs=1e-12)


def test_no_new_ratings_no_growth_is_identity(orc):
    tr, _ = planted()
    O = orc.Model(1200, 600, 8, 4, seed=77)
    O.load(tr.u, tr.i, tr.r)
    O.epoch(hp=HP)
    before = snapshot(O)
    O.add_ratings(1200, 600, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), HP, 3)
    for a, b in zip(before, snapshot(O)):
        assert np.array_equal(a, b)
    assert np.array_equal(O.u, tr.u)


def test_incremental_quality_close_to_scratch(orc):
    tr, te = planted()
    m0, n0 = 1000, 500
    old = (tr.u < m0) & (tr.i < n0)
    S = orc.Model(1200, 600, 8, 4, seed=77)
    S.load(tr.u, tr.i, tr.r)
    for _ in range(20):
        S.epoch(hp=HP)
    O = orc.Model(m0, n0, 8, 4, seed=77)
    O.load(tr.u[old], tr.i[old], tr.r[old])
    for _ in range(20):
        O.epoch(hp=HP)
    O.add_ratings(1200, 600, tr.u[~old], tr.i[~old], tr.r[~old], HP, 5)
    for _ in range(5):
        O.epoch(hp=HP)
    rs, ri = S.rmse(te.u, te.i, te.r), O.rmse(te.u, te.i, te.r)
    assert ri <= rs + 0.01, (ri, rs)
