"""Race check of the schedule on the device (bmf_check_disjoint; Section 3:
the blocks of one stratum share no user and no item).  On the epochs' own
schedule the count is zero for every SGD kernel; for other pairings of
block rows with block columns it is nonzero exactly when the ratings put
one user in two blocks of a stratum, which the test works out from the
ratings and the block sizes ceil(m / b), ceil(n / b).  The
BMF_CHECK_DISJOINT=1 epoch mode runs the check first and changes no
result."""
import sys

import numpy as np
import pytest

from paper_1907_07410_amd import synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def B():
    from paper_1907_07410_amd import binding
    return binding


def shares_a_row(u, i, m, n, b, pairing):
    """True when some stratum s holds two blocks (pairing[s, j], j) that
    both hold ratings of one user.  Items cannot be shared: the column fixes
    an item's block."""
    rb, cb = -(-m // b), -(-n // b)
    br, bc = u // rb, i // cb
    for s in range(b):
        inside = pairing[s][bc] == br
        pairs = np.unique(np.stack([u[inside], bc[inside]], 1), axis=0)
        if len(np.unique(pairs[:, 0])) < len(pairs):
            return True
    return False


def latin(b):
    return np.array([[(j + s) % b for j in range(b)] for s in range(b)], dtype=np.int32)


@pytest.mark.parametrize("m,n,k,b,kernel", [(1003, 500, 16, 4, 1), (1003, 500, 16, 4, 2), (2000, 1500, 64, 16, 2),
                                            (2000, 1500, 64, 16, 1), (600, 300, 200, 5, 0)])
def test_schedule_is_disjoint_and_broken_pairings_are_caught(B, m, n, k, b, kernel):
    rat = synth.random_coo(m, n, 30 * m, seed=m + b, dup=True)
    G = B.Model(m, n, k, b, sgd_kernel=kernel)
    G.load_ratings(rat.u, rat.i, rat.r)
    runs = G.plan_info()[0]
    log("shape", m, n, k, b, "kernel asked", kernel, "runs", runs)
    if kernel == 2:
        assert runs == 2  # the step plan's records are the ones checked
    assert G.check_disjoint() == 0
    assert G.check_disjoint(latin(b)) == 0
    rng = np.random.default_rng(b)
    # any permutation of the block rows per stratum is disjoint too
    perm = np.stack([rng.permutation(b) for _ in range(b)]).astype(np.int32)
    assert not shares_a_row(rat.u, rat.i, m, n, b, perm)
    assert G.check_disjoint(perm) == 0
    # two columns on one block row in one stratum: a race wherever both
    # blocks hold ratings of one user
    broken = latin(b)
    broken[1, 2] = broken[1, 3]
    want = shares_a_row(rat.u, rat.i, m, n, b, broken)
    got = G.check_disjoint(broken)
    log("broken pairing", got, "expected a race:", want)
    assert want and got > 0
    # every column on block row 0 in every stratum
    got = G.check_disjoint(np.zeros((b, b), np.int32))
    assert got > 0
    with pytest.raises(B.BmfError) as ex:
        bad = latin(b)
        bad[0, 0] = b
        G.check_disjoint(bad)
    assert ex.value.status == B.BMF_E_INVAL
    G.close()


def test_shared_row_without_shared_users_is_no_race(B):
    """Users of block row r rate only items of block column r: pairing every
    column with row 0 puts one non-empty block and b - 1 empty ones in a
    stratum, which share nothing, so the count stays zero."""
    m, n, b = 800, 400, 4
    rb, cb = m // b, n // b
    rng = np.random.default_rng(3)
    u = rng.integers(0, m, 20000).astype(np.int32)
    i = ((u // rb) * cb + rng.integers(0, cb, u.shape[0])).astype(np.int32)
    r = rng.integers(1, 6, u.shape[0]).astype(np.float32)
    for kernel in (1, 2):
        G = B.Model(m, n, 16, b, sgd_kernel=kernel)
        G.load_ratings(u, i, r)
        zeros = np.zeros((b, b), np.int32)
        assert not shares_a_row(u, i, m, n, b, zeros)
        assert G.check_disjoint(zeros) == 0
        assert G.check_disjoint() == 0
        G.close()


def test_check_mode_runs_before_every_epoch_and_changes_nothing(B, monkeypatch):
    m, n, k, b = 1003, 500, 16, 4
    rat = synth.random_coo(m, n, 20000, seed=7, dup=True)
    out = []
    for flag in ("0", "1"):
        monkeypatch.setenv("BMF_CHECK_DISJOINT", flag)
        G = B.Model(m, n, k, b, order_mode=1)
        G.load_ratings(rat.u, rat.i, rat.r)
        for _ in range(3):
            G.epoch(0.01, 0.02)
        out.append(G.get_factors())
        G.close()
    for a, c in zip(out[0][:4], out[1][:4]):
        assert np.array_equal(np.asarray(a).view(np.uint32), np.asarray(c).view(np.uint32))


def test_check_refuses_without_resident_ratings(B):
    G = B.Model(300, 200, 16, 4)
    with pytest.raises(B.BmfError) as ex:
        G.check_disjoint()
    assert ex.value.status == B.BMF_E_STATE
    G.close()
    rat = synth.random_coo(300, 200, 5000, seed=2, dup=True)
    G = B.Model(300, 200, 16, 4, out_of_core=True)
    G.load_ratings(rat.u, rat.i, rat.r)
    with pytest.raises(B.BmfError) as ex:
        G.check_disjoint()
    assert ex.value.status == B.BMF_E_STATE
    G.close()


def test_paper_grid_is_disjoint(B):
    """The paper's 3072 x 3072 grid on MovieLens-1M-sized data (2 users x 2
    items per block, most blocks empty or nearly): zero on the epochs'
    schedule, and a stratum that puts two columns a user rated on that
    user's block row is caught."""
    m, n, b = 6040, 3900, 3072
    rat = synth.random_coo(m, n, 1_000_000, seed=31, dup=True)
    G = B.Model(m, n, 13, b)
    G.load_ratings(rat.u, rat.i, rat.r)
    assert G.check_disjoint() == 0
    assert G.check_disjoint(latin(b)) == 0
    rb, cb = -(-m // b), -(-n // b)
    u0 = int(rat.u[0])
    cols = np.unique(rat.i[rat.u == u0] // cb)
    assert cols.size >= 2
    pairing = latin(b)
    pairing[0, cols[0]] = u0 // rb
    pairing[0, cols[1]] = u0 // rb
    got = G.check_disjoint(pairing)
    log("paper grid broken pairing", got)
    assert got > 0
    G.close()
