"""Step plans of the LDS-staged SGD kernel (host scheduler, no GPU).

A plan may reorder only ratings that share neither user nor item: the
update of Eqs 10-13 for rating (u, i) touches p_u, bu_u, q_i and bi_i alone,
so such ratings commute exactly and the plan's order gives the same result
as Algorithm 2's row-major order.  These tests check the plan's invariants
and replay both orders."""
import numpy as np
import pytest

B = pytest.importorskip("paper_1907_07410_amd.binding")


def make_block(rng, nu, ni, n, dup=0.02, zipf=1.1):
    """Ratings of one block in row-major order: Zipf-weighted users and
    items, a few duplicate (u, i) pairs."""
    wu = 1.0 / np.arange(1, nu + 1) ** zipf
    wi = 1.0 / np.arange(1, ni + 1) ** zipf
    u = rng.choice(nu, n, p=wu / wu.sum())
    i = rng.choice(ni, n, p=wi / wi.sum())
    pairs = np.unique(np.stack([u, i], 1), axis=0)
    nd = int(len(pairs) * dup)
    if nd:
        pairs = np.concatenate([pairs, pairs[rng.choice(len(pairs), nd)]])
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))  # stable: duplicates keep their order
    pairs = pairs[order]
    r = rng.integers(1, 11, len(pairs)).astype(np.float32) / 2
    return pairs[:, 0].astype(np.int32), pairs[:, 1].astype(np.int32), r


def check_plan(plan, u, i, r, cb, slots, chunk):
    n = len(u)
    meta = plan[:, :, 0]
    idx = plan[:, :, 3]
    il = meta & 0xFFFF
    sl = (meta >> 16) & 0x3FFF
    real = idx != 0xFFFFFFFF
    # empty records
    assert np.all(il[~real] == cb) and np.all(sl[~real] == slots)
    # every rating exactly once
    got = np.sort(idx[real].astype(np.int64))
    assert np.array_equal(got, np.arange(n))
    step_of = np.empty(n, np.int64)
    sidx = np.nonzero(real)
    step_of[idx[real]] = sidx[0]
    # record contents
    x = idx[real].astype(np.int64)
    assert np.array_equal(il[real], i[x])
    assert np.array_equal(plan[:, :, 2][real], u[x])
    assert np.array_equal(plan[:, :, 1][real].view(np.float32), r[x])
    # a step holds distinct users and distinct items
    for s in range(plan.shape[0]):
        m = real[s]
        xs = idx[s][m].astype(np.int64)
        assert len(set(u[xs])) == len(xs) and len(set(i[xs])) == len(xs)
    # per-user and per-item order kept
    for key in (u, i):
        o = np.lexsort((np.arange(n), key))
        same = key[o][1:] == key[o][:-1]
        assert np.all(step_of[o][1:][same] > step_of[o][:-1][same])
    # slots: one per user, FIRST / LAST flags, reuse distance
    slot_of = np.empty(n, np.int64)
    slot_of[x] = sl[real]
    first = np.zeros(n, bool)
    last = np.zeros(n, bool)
    first[x] = (meta[real] >> 30) & 1 == 1
    last[x] = (meta[real] >> 31) & 1 == 1
    starts = np.r_[True, u[1:] != u[:-1]]
    ends = np.r_[u[1:] != u[:-1], True]
    assert np.array_equal(first, starts) and np.array_equal(last, ends)
    assert np.all(slot_of < slots)
    runs = np.split(np.arange(n), np.nonzero(starts)[0][1:])
    uses = {}
    for run in runs:
        assert len(set(slot_of[run])) == 1
        uses.setdefault(int(slot_of[run[0]]), []).append((step_of[run].min() // chunk, step_of[run].max() // chunk))
    for iv in uses.values():
        iv.sort()
        for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
            assert b0 >= a1 + 3
    return step_of


def replay(u, i, r, order, k=4, lr=0.05, reg=0.02, seed=0):
    """FP64 SGD of Eqs 10-13 over the ratings in the given order."""
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 0.1, (u.max() + 1, k))
    Q = rng.normal(0, 0.1, (i.max() + 1, k))
    bu = np.zeros(u.max() + 1)
    bi = np.zeros(i.max() + 1)
    for x in order:
        a, b = u[x], i[x]
        e = r[x] - 3.0 - bu[a] - bi[b] - P[a] @ Q[b]
        pa, qb = P[a].copy(), Q[b].copy()
        P[a] = pa + lr * (e * qb - reg * pa)
        Q[b] = qb + lr * (e * pa - reg * qb)
        bu[a] += lr * (e - reg * bu[a])
        bi[b] += lr * (e - reg * bi[b])
    return P, Q, bu, bi


@pytest.mark.parametrize("seed,nu,ni,n,slots,chunk", [
    (0, 300, 120, 3000, 64, 16),
    (1, 2000, 400, 6000, 179, 16),
    (2, 50, 40, 1500, 8, 4),
    (3, 800, 60, 4000, 1, 16),
    (4, 5, 500, 2000, 4, 2),
])
def test_plan_invariants_and_replay(seed, nu, ni, n, slots, chunk):
    rng = np.random.default_rng(seed)
    u, i, r = make_block(rng, nu, ni, n)
    cb = ni + 3
    plan = B.block_plan(u, i, r, cb, slots, chunk)
    step_of = check_plan(plan, u, i, r, cb, slots, chunk)
    order = np.argsort(step_of, kind="stable")
    ref = replay(u, i, r, np.arange(len(u)))
    got = replay(u, i, r, order)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_plan_packs_independent_ratings():
    """With many light users the steps are nearly full: fewer than 0.4 steps
    per rating (a sequential walk would need 1)."""
    rng = np.random.default_rng(5)
    u, i, r = make_block(rng, 3000, 400, 6000)
    plan = B.block_plan(u, i, r, 400, 200, 16)
    check_plan(plan, u, i, r, 400, 200, 16)
    assert plan.shape[0] < 0.4 * len(u)


def test_plan_single_user_and_single_item_chains_are_sequential():
    # one user: every rating depends on the previous one
    u = np.zeros(50, np.int32)
    i = np.arange(50, dtype=np.int32)
    r = np.ones(50, np.float32)
    plan = B.block_plan(u, i, r, 64, 8, 16)
    assert plan.shape[0] == 50
    check_plan(plan, u, i, r, 64, 8, 16)
    # one item rated by many users: one chain as well
    u = np.arange(40, dtype=np.int32)
    i = np.full(40, 7, np.int32)
    plan = B.block_plan(u, i, np.ones(40, np.float32), 16, 40, 16)
    check_plan(plan, u, i, np.ones(40, np.float32), 16, 40, 16)
    assert plan.shape[0] == 40


def test_plan_empty_and_bad_input():
    plan = B.block_plan(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), 8, 4, 16)
    assert plan.shape == (0, 4, 4)
    with pytest.raises(B.BmfError) as ex:  # not in row-major order
        B.block_plan(np.array([1, 0], np.int32), np.array([0, 0], np.int32), np.ones(2, np.float32), 8, 4, 16)
    assert ex.value.status == B.BMF_E_INVAL
    with pytest.raises(B.BmfError) as ex:  # item outside the slice
        B.block_plan(np.array([0], np.int32), np.array([8], np.int32), np.ones(1, np.float32), 8, 4, 16)
    assert ex.value.status == B.BMF_E_RANGE


def _longest_chain(u, i):
    """Longest sequence of ratings t1 < t2 < ... in which each shares its
    user or its item with the one before (every pair examined)."""
    L = [1] * len(u)
    for t in range(len(u)):
        for s in range(t):
            if (u[s] == u[t] or i[s] == i[t]) and L[s] + 1 > L[t]:
                L[t] = L[s] + 1
    return max(L, default=0)


def test_chain_depth_matches_pairwise_search():
    """bmf_chain_depth (the dependency depth of a block under Algorithm 2's
    order) against an all-pairs search, and the plan never beats it."""
    rng = np.random.default_rng(8)
    for trial in range(40):
        nu, ni = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        n = int(rng.integers(0, 70))
        if n:
            u, i, r = make_block(rng, nu, ni, n)
        else:
            u, i, r = np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)
        d = B.chain_depth(u, i)
        assert d == _longest_chain(u.tolist(), i.tolist()), trial
        plan = B.block_plan(u, i, r, ni, 8, 16)
        assert plan.shape[0] >= max(d, -(-len(u) // 4))
    # one user's ratings and one item's ratings are chains of their length
    assert B.chain_depth(np.zeros(30, np.int32), np.arange(30, dtype=np.int32)) == 30
    assert B.chain_depth(np.arange(25, dtype=np.int32), np.full(25, 3, np.int32)) == 25
    assert B.chain_depth(np.arange(25, dtype=np.int32), np.arange(25, dtype=np.int32)) == 1
    with pytest.raises(B.BmfError):
        B.chain_depth(np.array([-1], np.int32), np.array([0], np.int32))
