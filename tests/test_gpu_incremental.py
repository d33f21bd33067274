"""Incremental data on the GPU (bmf_add_ratings) against the oracle's
add_ratings: grown rows, the new-ratings phase, the union's partition and
the epochs after it; untouched rows keep their bits; errors change
nothing."""
import numpy as np
import pytest

from paper_1907_07410_amd import synth

pytestmark = pytest.mark.gpu

HP = (0.01, 0.02) * 4


def planted(seed=5, m=1200, n=600, nnz=60000):
    rng = np.random.default_rng(seed)
    u, i = synth.sample_pairs_zipf(m, n, nnz, 0.6, 0.6, rng)
    r = synth.planted_values(u, i, m, n, 8, 0.4, 0.5, 3.5, "none", rng)
    return synth.split(synth.Ratings(u, i, r), 0.9, rng)


def pair(orc, m, n, k, b, u, i, r):
    from paper_1907_07410_amd import binding as B
    G = B.Model(m, n, k, b, seed=77, order_mode=0)
    G.load_ratings(u, i, r)
    O = orc.Model(m, n, k, b, seed=77, order_mode=0)
    O.load(u, i, r)
    return G, O


def diff(G, O):
    P, Q, bu, bi, mu = G.get_factors()
    assert P.shape == O.P.shape and Q.shape == O.Q.shape
    return max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(), np.abs(bi - O.bi).max())


@pytest.mark.parametrize("k,b", [(13, 4), (64, 8), (32, 2)])
def test_incremental_matches_oracle(orc, k, b):
    tr, te = planted()
    m0, n0 = 1000, 500
    old = (tr.u < m0) & (tr.i < n0)
    G, O = pair(orc, m0, n0, k, b, tr.u[old], tr.i[old], tr.r[old])
    for _ in range(3):
        G.epoch_hp(HP)
        O.epoch(hp=HP)
    G.add_ratings(1200, 600, tr.u[~old], tr.i[~old], tr.r[~old], HP, 2)
    O.add_ratings(1200, 600, tr.u[~old], tr.i[~old], tr.r[~old], HP, 2)
    d = diff(G, O)
    assert d <= 1e-4, d
    bp, perm = G.get_partition(len(tr))
    assert np.array_equal(bp, O.block_ptr) and np.array_equal(perm, O.perm)
    assert G.get_factors()[4] == pytest.approx(O.mu, abs=1e-12)
    for _ in range(2):
        G.epoch_hp(HP)
        O.epoch(hp=HP)
    assert diff(G, O) <= 1e-4
    assert G.epoch_count() == 7
    assert abs(G.rmse(te.u, te.i, te.r) - O.rmse(te.u, te.i, te.r)) <= 1e-4


def test_untouched_rows_keep_bits_and_growth_seeds_rows(orc):
    from paper_1907_07410_amd import binding as B
    tr, _ = planted()
    m0, n0 = 1000, 500
    old = (tr.u < m0) & (tr.i < n0)
    new = (tr.u >= m0) & (tr.i >= n0)
    G, _ = pair(orc, m0, n0, 16, 4, tr.u[old], tr.i[old], tr.r[old])
    for _ in range(2):
        G.epoch_hp(HP)
    P, Q, bu, bi, _mu = G.get_factors()
    G.add_ratings(1200, 600, tr.u[new], tr.i[new], tr.r[new], HP, 3)
    P2, Q2, bu2, bi2, _ = G.get_factors()
    assert np.array_equal(P2[:m0], P) and np.array_equal(Q2[:n0], Q)
    assert np.array_equal(bu2[:m0], bu) and np.array_equal(bi2[:n0], bi)
    # growth alone: new rows equal a fresh model's and the oracle's initial values
    H, _ = pair(orc, m0, n0, 16, 4, tr.u[old], tr.i[old], tr.r[old])
    H.add_ratings(1300, 650, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), HP, 1)
    F = B.Model(1300, 650, 16, 4, seed=77)
    Pf, Qf, _, _, _ = F.get_factors()
    Ph, Qh, buh, bih, _ = H.get_factors()
    Oi = orc.Model(1300, 650, 16, 4, seed=77)
    assert np.array_equal(Ph[m0:], Pf[m0:]) and np.array_equal(Qh[n0:], Qf[n0:])
    assert np.array_equal(Ph[m0:].astype(np.float64), Oi.P[m0:]) and np.array_equal(Qh[n0:].astype(np.float64), Oi.Q[n0:])
    assert not buh[m0:].any() and not bih[n0:].any()


def test_errors_change_nothing(orc):
    from paper_1907_07410_amd import binding as B
    tr, _ = planted()
    old = (tr.u < 1000) & (tr.i < 500)
    G, _ = pair(orc, 1000, 500, 16, 4, tr.u[old], tr.i[old], tr.r[old])
    G.epoch_hp(HP)
    before = G.get_factors()
    bad_u = np.array([5, 1300], np.int32)
    ok_i = np.array([1, 2], np.int32)
    rr = np.array([3.0, 4.0], np.float32)
    with pytest.raises(B.BmfError):
        G.add_ratings(1200, 600, bad_u, ok_i, rr, HP, 1)  # user beyond m_new
    with pytest.raises(B.BmfError):
        G.add_ratings(900, 600, ok_i, ok_i, rr, HP, 1)  # shrinks
    with pytest.raises(B.BmfError):
        G.add_ratings(1200, 600, ok_i, ok_i, np.array([3.0, np.nan], np.float32), HP, 1)
    with pytest.raises(B.BmfError):
        G.add_ratings(1200, 600, ok_i, ok_i, rr, HP, -1)
    after = G.get_factors()
    for a, b in zip(before, after):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert G.epoch_count() == 1
