"""Pins of the oracle's training loop (Algorithm 1): epochs run until the
training RMSE improves by less than delta over the previous epoch, at most
the maximum number of steps.

The rule is checked against a trajectory recorded one epoch at a time on a
separate model: the stopping epoch is the first whose improvement falls
under delta, every earlier epoch improved by at least delta, and the fitted
factors are bit-identical to those of the trajectory at that epoch.  Special
cases: zero steps, a delta no improvement reaches (one epoch), a negative
delta no change reaches (all steps), and larger deltas never run longer."""
import numpy as np
import pytest

from paper_1907_07410_amd import configs, synth


def make(orc, prob, k=13, b=4):
    O = orc.Model(prob.m, prob.n, k, b, seed=1001, order_mode=0)
    O.load(prob.train.u, prob.train.i, prob.train.r)
    return O


@pytest.fixture(scope="module")
def small():
    return configs.PAPER_ML1M.generate(1, scale=0.1)


def trajectory(orc, prob, steps):
    O = make(orc, prob)
    out = [O.rmse()]
    snaps = [None]
    for _ in range(steps):
        O.epoch(hp=configs.PAPER_HP)
        out.append(O.rmse())
        snaps.append((O.P.copy(), O.Q.copy(), O.bu.copy(), O.bi.copy()))
    return np.array(out), snaps


def test_stopping_rule_against_trajectory(orc, small):
    rm, snaps = trajectory(orc, small, 80)
    imp = rm[:-1] - rm[1:]
    for delta in (1e-2, 1e-3, 1e-4):
        O = make(orc, small)
        e, r = O.fit(configs.PAPER_HP, 80, delta)
        assert 1 <= e <= 80
        assert np.all(imp[: e - 1] >= delta)
        assert e == 80 or imp[e - 1] < delta
        assert r == rm[e]
        P, Q, bu, bi = snaps[e]
        assert np.array_equal(O.P, P) and np.array_equal(O.Q, Q)
        assert np.array_equal(O.bu, bu) and np.array_equal(O.bi, bi)


def test_fit_special_cases(orc, small):
    O = make(orc, small)
    r0 = O.rmse()
    assert O.fit(configs.PAPER_HP, 0, 1e-4) == (0, r0)
    assert O.epoch_no == 0
    O = make(orc, small)
    e, r = O.fit(configs.PAPER_HP, 50, 1e9)
    assert e == 1 and O.epoch_no == 1
    O = make(orc, small)
    e, r = O.fit(configs.PAPER_HP, 7, -1e9)
    assert e == 7 and O.epoch_no == 7


def test_larger_delta_stops_no_later(orc, small):
    runs = []
    for delta in (1e-5, 1e-4, 1e-3, 1e-2):
        runs.append(make(orc, small).fit(configs.PAPER_HP, 200, delta)[0])
    assert runs == sorted(runs, reverse=True)
    # Training under the paper's pairs does improve for a while.
    assert runs[1] > 5


def test_paper_pairs_reduce_training_rmse(orc):
    prob = synth.Problem(300, 200, synth.random_coo(300, 200, 6000, seed=3), None)
    O = make(orc, prob, k=13, b=2)
    r0 = O.rmse()
    e, r = O.fit(configs.PAPER_HP, 30, 1e-4)
    assert r < r0


def test_diverging_fit_stops(orc, small):
    """Rates far too large blow the factors up; the loop ends at the first
    epoch whose RMSE is not a number instead of running every step."""
    O = make(orc, small)
    e, r = O.fit((5.0, 0.0) * 4, 60, 1e-4)
    assert e < 60 and not np.isfinite(r)
