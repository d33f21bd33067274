"""Out-of-core training (BMF_OPT_OUT_OF_CORE): ratings stay in pinned host
memory and each stratum is copied to the device while the previous one runs.

* the host partition equals the oracle's (ragged grids, duplicates, empty
  blocks);
* with the same SGD kernel the factors are bit-identical to a resident load
  (mu = 0, seeded stratum order; planned, 16-lane and 64-lane reference
  kernels);
* with mu from the data, mu equals the oracle's FP64 mean and one epoch is
  within 1e-4 of the oracle;
* RMSE, loss and the stopping-rule fit agree with the resident path;
* misuse is refused."""
import numpy as np
import pytest

from paper_1907_07410_amd import configs, synth

pytestmark = pytest.mark.gpu

HP = (0.01, 0.02) * 4


def data(seed=3, m=1500, n=700, nnz=40000, dup=False):
    if dup:
        return synth.random_coo(m, n, nnz, seed, dup=True)
    rng = np.random.default_rng(seed)
    u, i = synth.sample_pairs_zipf(m, n, nnz, 0.8, 0.8, rng)
    r = synth.planted_values(u, i, m, n, 8, 0.4, 0.5, 3.5, "half", rng)
    return synth.Ratings(u, i, r)


def model(B, m, n, k, b, ooc, kernel=None, mu_mode=None, order_mode=1):
    return B.Model(m, n, k, b, seed=11, order_mode=order_mode, order_seed=21, mu_mode=mu_mode, sgd_kernel=kernel,
                   out_of_core=ooc)


@pytest.mark.parametrize("m,n,b,dup", [(1500, 700, 8, False), (1000, 999, 7, True), (37, 1200, 16, False)])
def test_host_partition_matches_oracle(orc, m, n, b, dup):
    from paper_1907_07410_amd import binding as B
    d = data(m=m, n=n, nnz=min(30000, m * n // 3), dup=dup)
    G = model(B, m, n, 16, b, True)
    G.load_ratings(d.u, d.i, d.r)
    bp, perm = G.get_partition(len(d.u))
    obp, operm = orc.partition(m, n, b, d.u, d.i)
    assert np.array_equal(bp, obp) and np.array_equal(perm, operm)


@pytest.mark.parametrize("order_mode", [0, 1])
@pytest.mark.parametrize("k,b,kernel", [(64, 8, None), (64, 8, 1), (13, 128, None), (32, 4, 2), (200, 4, None),
                                        (32, 12, None), (16, 20, 1)])
def test_bit_identical_to_resident(k, b, kernel, order_mode):
    """Strata travel in groups of up to eight per ring buffer: in the epoch's
    order, so with the identity order a group is one copy and with the seeded
    order several; grids of 12 and 20 end on a partial group."""
    from paper_1907_07410_amd import binding as B
    d = data()
    out = []
    for ooc in (False, True):
        G = model(B, 1500, 700, k, b, ooc, kernel=kernel, mu_mode=1, order_mode=order_mode)
        G.load_ratings(d.u, d.i, d.r)
        for _ in range(3):
            G.epoch_hp(HP)
        out.append(G.get_factors()[:4])
    for a, c in zip(*out):
        assert np.array_equal(a, c)


def test_mean_and_epoch_against_oracle(orc):
    from paper_1907_07410_amd import binding as B
    d = data()
    G = model(B, 1500, 700, 32, 8, True, order_mode=0)
    G.load_ratings(d.u, d.i, d.r)
    O = orc.Model(1500, 700, 32, 8, seed=11, order_mode=0)
    O.load(d.u, d.i, d.r)
    assert G.get_factors()[4] == O.mu
    G.epoch_hp(HP)
    O.epoch(hp=HP)
    P, Q, bu, bi, _ = G.get_factors()
    assert max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(), np.abs(bi - O.bi).max()) <= 1e-4


def test_rmse_loss_fit_match_resident():
    from paper_1907_07410_amd import binding as B
    d = data()
    res = []
    for ooc in (False, True):
        G = model(B, 1500, 700, 16, 8, ooc, mu_mode=1)
        G.load_ratings(d.u, d.i, d.r)
        e, r = G.fit(configs.PAPER_HP, 40, 1e-4)
        res.append((e, r, G.rmse(), G.loss(hp=HP)))
    (e0, r0, t0, l0), (e1, r1, t1, l1) = res
    assert e0 == e1
    assert abs(r0 - r1) <= 1e-12 * max(1.0, r0) and abs(t0 - t1) <= 1e-12 * max(1.0, t0)
    assert abs(l0 - l1) <= 1e-9 * max(1.0, abs(l0))


def test_misuse_refused():
    import torch
    from paper_1907_07410_amd import binding as B
    d = data()
    G = model(B, 1500, 700, 16, 8, True)
    with pytest.raises(B.BmfError):
        G.load_ratings_dev(torch.from_numpy(d.u).cuda(), torch.from_numpy(d.i).cuda(), torch.from_numpy(d.r).cuda())
    G.load_ratings(d.u, d.i, d.r)
    with pytest.raises(B.BmfError) as ex:
        G.add_ratings(1600, 700, d.u[:5], d.i[:5], d.r[:5], HP, 1)
    assert ex.value.status == B.BMF_E_STATE
    G.set_option(B.OPT_SGD_KERNEL, 1)  # the load laid out planned steps
    with pytest.raises(B.BmfError) as ex:
        G.epoch_hp(HP)
    assert ex.value.status == B.BMF_E_STATE
    G.set_option(B.OPT_SGD_KERNEL, 0)
    G.epoch_hp(HP)
    bad = d.u.copy()
    bad[7] = 1500
    with pytest.raises(B.BmfError) as ex:
        G.load_ratings(bad, d.i, d.r)
    assert ex.value.status == B.BMF_E_RANGE
    # back to resident on the same context
    G.set_option(B.OPT_OUT_OF_CORE, 0)
    G.load_ratings(d.u, d.i, d.r)
    G.epoch_hp(HP)
