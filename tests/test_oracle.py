"""Pins for the FP64 oracle: worked examples, closed forms, invariants and
brute force on tiny inputs.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

from paper_1907_07410_amd import configs, synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------- RNG / init
def test_splitmix64_published_vector(orc):
    g = _gold("splitmix64.json")
    got = [orc.splitmix64(g["seed"], j) for j in range(len(g["outputs"]))]
    assert got == [int(x) for x in g["outputs"]]


def test_init_values_exact_in_fp32(orc):
    m, n, k = 37, 23, 13
    M = orc.Model(m, n, k, 3, seed=99)
    for A in (M.P, M.Q):
        assert np.all(A >= -0.125) and np.all(A < 0.125)
        assert np.array_equal(A.astype(np.float32).astype(np.float64), A)
        # 24-bit grid: value * 2^26 is an integer
        assert np.array_equal(np.round(A * 2**26), A * 2**26)
    assert np.all(M.bu == 0) and np.all(M.bi == 0)
    # the two tensors come from different streams
    assert not np.array_equal(M.P[:10, :], M.Q[:10, :])
    # counter-based: an entry depends only on (seed, tensor, row, factor)
    assert M.P[5, 7] == orc.init_value(99, 1, 5, k, 7)
    assert M.Q[22, 12] == orc.init_value(99, 2, 22, k, 12)


def test_bf16_rounding_cases(orc):
    for c in _gold("bf16_rne.json")["cases"]:
        assert orc.bf16_round(c["x"]) == c["bf16"], c


def test_bf16_rounding_of_arrays(orc):
    cases = _gold("bf16_rne.json")["cases"]
    x = np.array([c["x"] for c in cases], dtype=np.float32).reshape(1, -1)
    y = orc.bf16_round_array(x)
    assert y.shape == x.shape and y.dtype == np.float32
    assert [float(v) for v in y[0]] == [c["bf16"] for c in cases]
    # every element as the one-value form rounds it; a BF16 value has at
    # most 8 significant bits and lies within half a BF16 step (2^-8
    # relative) of the input
    r = np.random.default_rng(5).normal(0, 3, (7, 33)).astype(np.float32)
    y = orc.bf16_round_array(r)
    assert all(y.flat[t] == orc.bf16_round(float(r.flat[t])) for t in range(r.size))
    assert np.all(y.view(np.uint32) & 0xFFFF == 0)
    assert np.all(np.abs(y.astype(np.float64) - r) <= 2.0 ** -8 * np.abs(r.astype(np.float64)))


# ------------------------------------------------------------ update rules
def _single(orc, g, form):
    inp = g["inputs"]
    M = orc.Model(1, 1, 2, 1, seed=1)
    M.load([0], [0], [inp["r"]])
    M.set_factors(np.array([inp["p"]]), np.array([inp["q"]]), [inp["bu"]], [inp["bi"]], inp["mu"])
    M.epoch(inp["lr"], inp["reg"], gauss_seidel=form == "gauss_seidel", alg2_literal=form == "alg2_literal")
    return M


@pytest.mark.parametrize("form", ["simultaneous", "gauss_seidel", "alg2_literal"])
def test_single_rating_worked_example(orc, form):
    g = _gold("single_update.json")
    M = _single(orc, g, form)
    want = g[form]
    assert M.bu[0] == pytest.approx(want["bu"], abs=1e-15)
    assert M.bi[0] == pytest.approx(want["bi"], abs=1e-15)
    np.testing.assert_allclose(M.P[0], want["p"], atol=1e-15, rtol=0)
    np.testing.assert_allclose(M.Q[0], want["q"], atol=1e-15, rtol=0)


def test_per_name_hyperparameters_route_to_their_parameter(orc):
    """Each (alpha, beta) pair of Eqs 10-13 moves only its own parameter."""
    g = _gold("single_update.json")["inputs"]
    base = np.array([g["lr"], g["reg"]] * 4)
    for which in range(4):
        hp = np.zeros(8)
        hp[2 * which:2 * which + 2] = base[2 * which:2 * which + 2]
        M = orc.Model(1, 1, 2, 1, seed=1)
        M.load([0], [0], [g["r"]])
        M.set_factors(np.array([g["p"]]), np.array([g["q"]]), [g["bu"]], [g["bi"]], g["mu"])
        M.epoch(hp=hp)
        moved = [not np.array_equal(M.P[0], g["p"]), not np.array_equal(M.Q[0], g["q"]),
                 M.bu[0] != g["bu"], M.bi[0] != g["bi"]]
        assert moved == [j == which for j in range(4)]


def test_bias_dynamics_closed_form(orc):
    """One rating, zero factors, no global mean: the factors stay exactly
    zero and bu_t = bi_t = b* (1 - (1 - lr (2 + reg))^t), b* = r / (2 + reg)."""
    r, lr, reg = 4.0, 0.01, 0.02
    M = orc.Model(1, 1, 3, 1, seed=5, mu_mode=1)
    M.load([0], [0], [r])
    M.set_factors(np.zeros((1, 3)), np.zeros((1, 3)), [0.0], [0.0], 0.0)
    bstar = r / (2 + reg)
    assert bstar == pytest.approx(1.98019801980198, abs=1e-13)
    for t in range(1, 301):
        M.epoch(lr, reg)
        want = bstar * (1 - (1 - lr * (2 + reg)) ** t)
        assert M.bu[0] == pytest.approx(want, abs=1e-12)
        assert M.bi[0] == pytest.approx(want, abs=1e-12)
        assert np.all(M.P == 0) and np.all(M.Q == 0)


# --------------------------------------------------------------- partition
def test_partition_paper_block_extents(orc):
    """Section 5: 6040 users on an 8 x 8 grid gives 755-row blocks; 486
    columns per block fits ceil(n / 8) for n in 3881..3888."""
    m, n, b = 6040, 3885, 8
    u = np.array([754, 755, 6039, 0, 0], dtype=np.int32)
    i = np.array([485, 486, 3884, 0, 3884], dtype=np.int32)
    bp, perm = orc.partition(m, n, b, u, i)
    sizes = np.diff(bp).reshape(b, b)
    assert sizes[0, 0] == 2       # (754, 485) and (0, 0)
    assert sizes[1, 1] == 1       # (755, 486)
    assert sizes[7, 7] == 1       # (6039, 3884)
    assert sizes[0, 7] == 1       # (0, 3884)
    assert math.ceil(m / b) == 755 and all(math.ceil(nn / b) == 486 for nn in range(3881, 3889))


def _brute_partition(m, n, b, u, i):
    rb, cb = -(-m // b), -(-n // b)
    blk = (u.astype(np.int64) // rb) * b + (i.astype(np.int64) // cb)
    t = np.arange(u.shape[0])
    order = np.lexsort((t, i, u, blk))
    bp = np.zeros(b * b + 1, dtype=np.int64)
    np.add.at(bp, blk + 1, 1)
    return np.cumsum(bp), order.astype(np.int32)


@pytest.mark.parametrize("m,n,b,nnz,dup", [(7, 5, 3, 20, True), (50, 40, 4, 300, False), (9, 100, 16, 200, True),
                                           (100, 3, 8, 250, True), (1, 1, 1, 5, True), (30, 30, 1, 0, False)])
def test_partition_matches_brute_force(orc, m, n, b, nnz, dup):
    rat = synth.random_coo(m, n, nnz, seed=m * 7 + b, dup=dup) if nnz else synth.Ratings(
        np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    bp, perm = orc.partition(m, n, b, rat.u, rat.i)
    bp2, perm2 = _brute_partition(m, n, b, rat.u, rat.i)
    assert np.array_equal(bp, bp2)
    assert np.array_equal(perm, perm2)


# ---------------------------------------------------------------- schedule
@pytest.mark.parametrize("b", [1, 2, 3, 6, 8, 64])
def test_strata_form_latin_square(orc, b):
    for mode in (0, 1):
        for e in range(3):
            order = orc.schedule(b, 2001, e, mode)
            assert sorted(order.tolist()) == list(range(b))
            seen = np.zeros((b, b), dtype=int)
            for s in order:
                rows = [(j + s) % b for j in range(b)]
                assert sorted(rows) == list(range(b))  # every block row once per stratum
                for j in range(b):
                    seen[(j + s) % b, j] += 1
            assert np.all(seen == 1)  # every block once per epoch (Section 3)
        if mode == 0:
            assert orc.schedule(b, 2001, 5, 0).tolist() == list(range(b))


def test_paper_stratum_order_diagonal_then_below():
    """Section 3 (parallel BMF): the diagonal blocks form the first parallel
    step, the blocks just below them the second, columns wrap."""
    b = 6
    s0 = {((j + 0) % b, j) for j in range(b)}
    s1 = {((j + 1) % b, j) for j in range(b)}
    assert s0 == {(d, d) for d in range(b)}
    assert s1 == {(d + 1, d) for d in range(b - 1)} | {(0, b - 1)}


def test_seeded_order_depends_on_seed_and_epoch(orc):
    a = orc.schedule(64, 11, 0, 1)
    assert not np.array_equal(a, orc.schedule(64, 11, 1, 1))
    assert not np.array_equal(a, orc.schedule(64, 12, 0, 1))
    assert np.array_equal(a, orc.schedule(64, 11, 0, 1))


def test_blocks_of_a_stratum_touch_disjoint_users_and_items(orc):
    p = configs.TINY.generate(1)
    m, n, b = p.m, p.n, 4
    bp, perm = orc.partition(m, n, b, p.train.u, p.train.i)
    for s in range(b):
        us, its = set(), set()
        for j in range(b):
            blk = ((j + s) % b) * b + j
            sel = perm[bp[blk]:bp[blk + 1]]
            bu_set, bi_set = set(p.train.u[sel].tolist()), set(p.train.i[sel].tolist())
            assert not (us & bu_set) and not (its & bi_set)
            us |= bu_set
            its |= bi_set


# ------------------------------------------------------------ epoch driver
def test_epoch_visits_every_rating_once_in_schedule_order(orc):
    """An epoch equals applying the single-rating update to every rating,
    one at a time, in the order: strata in the epoch's order, blocks
    ((j+s) mod b, j) for j = 0..b-1, ratings (u, i, input index) inside a
    block.  The order here is rebuilt independently of the oracle's
    partition; the single-rating step is the one pinned above."""
    m, n, b, k = 11, 9, 3, 4
    rat = synth.random_coo(m, n, 60, seed=3, dup=True)
    A = orc.Model(m, n, k, b, seed=17, order_mode=1, order_seed=5)
    A.load(rat.u, rat.i, rat.r)
    order = A.order(0)
    A.epoch(0.05, 0.03)
    rb, cb = -(-m // b), -(-n // b)
    blk = (rat.u // rb) * b + rat.i // cb
    seq = []
    for s in order:
        for j in range(b):
            want = ((j + s) % b) * b + j
            idx = np.nonzero(blk == want)[0]
            idx = idx[np.lexsort((idx, rat.i[idx], rat.u[idx]))]
            seq.extend(idx.tolist())
    assert sorted(seq) == list(range(60))
    B = orc.Model(m, n, k, 1, seed=17)
    mu = A.mu
    for t in seq:
        B.load(rat.u[t:t + 1], rat.i[t:t + 1], rat.r[t:t + 1])
        B.mu = mu
        B.epoch(0.05, 0.03)
    assert np.array_equal(A.P, B.P) and np.array_equal(A.Q, B.Q)
    assert np.array_equal(A.bu, B.bu) and np.array_equal(A.bi, B.bi)


def test_thread_count_invariance(orc):
    p = configs.TINY.generate(2)
    res = []
    for T in (1, 2, 3, 4):
        M = orc.Model(p.m, p.n, 16, 4, seed=7, order_mode=1)
        M.load(p.train.u, p.train.i, p.train.r)
        for _ in range(2):
            M.epoch(0.01, 0.02, threads=T)
        res.append((M.P.copy(), M.Q.copy(), M.bu.copy(), M.bi.copy()))
    for r in res[1:]:
        for a, b in zip(res[0], r):
            assert np.array_equal(a, b)


def test_one_block_is_plain_mf_order(orc):
    """b = 1 is plain sequential SGD over the ratings in row-major order
    (Section 3's limiting case): the single block holds every rating in
    (u, i, input index) order."""
    rat = synth.random_coo(20, 15, 80, seed=4, dup=True)
    bp, perm = orc.partition(20, 15, 1, rat.u, rat.i)
    assert bp.tolist() == [0, 80]
    assert np.array_equal(perm, np.lexsort((np.arange(80), rat.i, rat.u)))


# --------------------------------------------------------------- evaluation
def test_rmse_closed_form_zero_factors(orc):
    p = configs.TINY.generate(3)
    M = orc.Model(p.m, p.n, 16, 4, seed=1)
    M.load(p.train.u, p.train.i, p.train.r)
    M.set_factors(np.zeros_like(M.P), np.zeros_like(M.Q), np.zeros(p.m), np.zeros(p.n))
    r = p.train.r.astype(np.float64)
    mu = math.fsum(r) / r.shape[0]
    assert M.mu == pytest.approx(mu, rel=1e-14)
    want = math.sqrt(math.fsum((r - mu) ** 2) / r.shape[0])
    assert M.rmse() == pytest.approx(want, rel=1e-12)


def test_loss_closed_form_zero_factors(orc):
    rat = synth.random_coo(6, 5, 20, seed=9, dup=True)
    M = orc.Model(6, 5, 3, 2, seed=1)
    M.load(rat.u, rat.i, rat.r)
    bu = np.linspace(-0.2, 0.3, 6)
    bi = np.linspace(0.1, -0.4, 5)
    M.set_factors(np.zeros((6, 3)), np.zeros((5, 3)), bu, bi)
    hp = np.array([0.0, 0.5, 0.0, 0.25, 0.0, 0.125, 0.0, 0.0625])
    terms = []
    for t in range(20):
        e = float(rat.r[t]) - M.mu - bu[rat.u[t]] - bi[rat.i[t]]
        terms += [e * e, 0.125 * bu[rat.u[t]] ** 2, 0.0625 * bi[rat.i[t]] ** 2]
    assert M.loss(hp=hp) == pytest.approx(math.fsum(terms), rel=1e-12)


def test_loss_worked_example(orc):
    """Eq 9 with non-zero factors and biases, four different betas and
    alphas that must not enter (tests/golden/loss_worked.json, worked by
    hand): a swapped alpha/beta, a dropped square or a missing penalty term
    changes the value."""
    g = _gold("loss_worked.json")
    inp = g["inputs"]
    rat = np.array(inp["ratings"])
    M = orc.Model(2, 2, 2, 1, seed=1)
    M.load(rat[:, 0].astype(np.int32), rat[:, 1].astype(np.int32), rat[:, 2].astype(np.float32))
    M.set_factors(np.array(inp["P"]), np.array(inp["Q"]), inp["bu"], inp["bi"], inp["mu"])
    h = inp["hp"]
    hp = [h["alpha_p"], h["beta_p"], h["alpha_q"], h["beta_q"], h["alpha_bu"], h["beta_bu"], h["alpha_bi"],
          h["beta_bi"]]
    assert M.loss(hp=hp) == pytest.approx(g["loss"], rel=1e-13)
    # each rating's term alone (the loss is a sum over observed ratings)
    for t, want in enumerate(g["terms"]):
        M.load(rat[t:t + 1, 0].astype(np.int32), rat[t:t + 1, 1].astype(np.int32),
               rat[t:t + 1, 2].astype(np.float32))
        M.mu = inp["mu"]
        assert M.loss(hp=hp) == pytest.approx(want, rel=1e-13)


def test_alg2_literal_equals_simultaneous_when_the_crossed_terms_vanish(orc):
    """Algorithm 2 as printed differs from Eqs 10-13 only through the
    crossed bias penalties and the factor order: with no bias penalty and
    no item-factor step the three forms give the same bits."""
    rat = synth.random_coo(9, 7, 80, seed=8, dup=True)
    out = []
    for form in ("simultaneous", "gauss_seidel", "alg2_literal"):
        M = orc.Model(9, 7, 3, 2, seed=3)
        M.load(rat.u, rat.i, rat.r)
        hp = [0.05, 0.02, 0.0, 0.02, 0.04, 0.0, 0.03, 0.0]
        for _ in range(3):
            M.epoch(hp=hp, gauss_seidel=form == "gauss_seidel", alg2_literal=form == "alg2_literal")
        out.append((M.P, M.Q, M.bu, M.bi))
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)


def test_noise_free_planted_matrix_is_recovered(orc):
    """r = 3.5 + u.v exactly (no noise, no rounding), k >= planted rank,
    no regularisation: the training RMSE goes to ~0."""
    m, n, rank = 60, 50, 3
    rng = np.random.default_rng(0)
    u, i = synth.sample_pairs_uniform(m, n, 1800, rng)
    r = synth.planted_values(u, i, m, n, rank, 0.5, 0.0, 3.5, "none", rng)
    M = orc.Model(m, n, 6, 4, seed=3, mu_mode=1)
    M.load(u, i, r)
    M.set_factors(M.P * 4, M.Q * 4, M.bu, M.bi, 3.5)
    first = M.rmse()
    for _ in range(600):
        M.epoch(0.05, 0.0)
    assert first > 0.2
    assert M.rmse() < 2e-3


def test_loss_non_increasing_at_small_lr(orc):
    p = configs.TINY.generate(4)
    M = orc.Model(p.m, p.n, 16, 4, seed=9, order_mode=1)
    M.load(p.train.u, p.train.i, p.train.r)
    prev = M.loss(1e-3, 0.02)
    for _ in range(15):
        M.epoch(1e-3, 0.02)
        cur = M.loss(1e-3, 0.02)
        assert cur <= prev
        prev = cur


def test_block_count_does_not_change_quality(orc):
    """Section 5: the block decomposition leaves the quality unchanged
    (Table 1's SVD and block rows differ by at most 0.004 RMSE)."""
    p = configs.TINY.generate(5)
    out = {}
    for b in (1, 4, 8):
        M = orc.Model(p.m, p.n, 16, b, seed=11, order_mode=1)
        M.load(p.train.u, p.train.i, p.train.r)
        for _ in range(20):
            M.epoch(0.01, 0.02)
        out[b] = M.rmse()
    assert abs(out[4] - out[1]) <= 0.005 and abs(out[8] - out[1]) <= 0.005


# -------------------------------------------------------------------- top-K
def test_topk_matches_brute_force(orc):
    rng = np.random.default_rng(1)
    m, n, k, K = 7, 300, 5, 20
    P, Q = rng.normal(size=(m, k)), rng.normal(size=(n, k))
    bu, bi = rng.normal(size=m), rng.normal(size=n)
    users = np.array([0, 3, 6, 3])
    items, scores = orc.topk_dense(P, Q, bu, bi, 3.5, users, K)
    for row, u in enumerate(users):
        s = np.array([3.5 + bu[u] + bi[j] + sum(P[u, f] * Q[j, f] for f in range(k)) for j in range(n)])
        want = sorted(range(n), key=lambda j: (-s[j], j))[:K]
        assert items[row].tolist() == want
        np.testing.assert_allclose(scores[row], s[want], rtol=0, atol=1e-12)


def test_topk_ties_go_to_smaller_item(orc):
    k, n = 3, 10
    Q = np.tile(np.array([[0.5, -0.25, 0.125]]), (n, 1))
    bi = np.zeros(n)
    P = np.array([[1.0, 1.0, 1.0]])
    items, scores = orc.topk_dense(P, Q, [0.0], bi, 0.0, [0], 4)
    assert items[0].tolist() == [0, 1, 2, 3]
    bi[7] = 1e-9
    items, _ = orc.topk_dense(P, Q, [0.0], bi, 0.0, [0], 4)
    assert items[0].tolist() == [7, 0, 1, 2]


def test_topk_k_larger_than_n_pads(orc):
    items, scores = orc.topk_dense(np.ones((1, 2)), np.ones((3, 2)), [0.0], [0.0, 0.1, 0.2], 0.0, [0], 5)
    assert items[0].tolist() == [2, 1, 0, -1, -1]
    assert np.isinf(scores[0, 3]) and scores[0, 3] < 0


def test_topk_vec_matches_brute_force(orc):
    """Ranking of an explicit user vector (a folded-in user): every item's
    score mu + bu + bi_i + p . q_i, best first, ties to the smaller id,
    checked against a full Python sort of scores summed with math.fsum."""
    rng = np.random.default_rng(12)
    n, k, K = 250, 6, 30
    Q = rng.normal(size=(n, k))
    bi = rng.normal(size=n)
    bi[17] = bi[3]
    Q[17] = Q[3]  # an exact tie: 3 must come first if it makes the list
    p = rng.normal(size=k)
    bu = 0.37
    items, scores = orc.topk_vec(p, bu, Q, bi, 2.5, K)
    s = [math.fsum([2.5, bu, bi[j]] + [p[f] * Q[j, f] for f in range(k)]) for j in range(n)]
    want = sorted(range(n), key=lambda j: (-s[j], j))[:K]
    assert items.tolist() == want
    np.testing.assert_allclose(scores, [s[j] for j in want], rtol=0, atol=1e-12)
    # K beyond n pads with -1 / -inf
    items, scores = orc.topk_vec(p[:2], bu, Q[:4, :2], bi[:4], 0.0, 6)
    assert sorted(items[:4].tolist()) == [0, 1, 2, 3] and items[4:].tolist() == [-1, -1]
    assert np.all(np.isneginf(scores[4:]))


def test_topk_vec_equals_topk_of_the_same_user_row(orc):
    """A user vector ranked alone equals the same vector ranked as row u of
    a factor table, bit for bit."""
    rng = np.random.default_rng(13)
    m, n, k, K = 5, 400, 9, 50
    P, Q = rng.normal(size=(m, k)), rng.normal(size=(n, k))
    bu, bi = rng.normal(size=m), rng.normal(size=n)
    for u in range(m):
        ti, ts = orc.topk_dense(P, Q, bu, bi, 3.25, [u], K)
        vi, vs = orc.topk_vec(P[u], bu[u], Q, bi, 3.25, K)
        assert np.array_equal(ti[0], vi) and np.array_equal(ts[0], vs)


# ------------------------------------------------------------------ fold-in
def test_foldin_approaches_ridge_solution(orc):
    """With items frozen the per-rating objective sum_j 1/2 (e_j^2 +
    beta (|p|^2 + bu^2)) is a ridge problem in (p, bu); many passes at a
    small step approach its closed-form solution."""
    rng = np.random.default_rng(2)
    n, k, cnt = 40, 4, 12
    Q = rng.normal(0, 0.5, size=(n, k))
    bi = rng.normal(0, 0.3, size=n)
    items = rng.choice(n, size=cnt, replace=False).astype(np.int32)
    r = rng.uniform(1, 5, size=cnt).astype(np.float32)
    mu, reg = 3.0, 0.05
    p, bu = orc.foldin(Q, bi, mu, items, r, passes=20000, lr=2e-3, reg=reg)
    X = np.hstack([Q[items], np.ones((cnt, 1))])
    y = r.astype(np.float64) - mu - bi[items]
    w = np.linalg.solve(X.T @ X + cnt * reg * np.eye(k + 1), X.T @ y)
    np.testing.assert_allclose(np.append(p, bu), w, atol=5e-3)


def test_foldin_first_step_by_hand(orc):
    Q = np.array([[0.5, -1.0]])
    bi = np.array([0.25])
    p, bu = orc.foldin(Q, bi, 3.0, [0], [4.0], passes=1, lr=0.1, reg=0.5)
    # p = 0, bu = 0 -> err = 4 - 3 - 0 - 0.25 - 0 = 0.75
    assert bu == pytest.approx(0.075, abs=1e-15)
    np.testing.assert_allclose(p, [0.0375, -0.075], atol=1e-15)
