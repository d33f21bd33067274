"""Host logic of the top-K plan (bmf_debug_topk_plan, no device): the
threshold rank, the candidate buffer's size against the order statistics of
the sample, the filter's item splits, and the workspace limits the header
states for the no-allocation entry point.  Pinned against scipy's Poisson
and Beta distributions, not against the library's own formulas."""
import numpy as np
import pytest
from scipy import stats

SHAPES = [  # (items, factors, K, precision)
    (100_000, 128, 100, 0), (100_000, 128, 100, 1), (17_800, 128, 100, 0), (17_800, 128, 100, 1),
    (27_000, 64, 100, 0), (27_000, 64, 100, 1), (20_000, 64, 100, 1), (1_000_000, 128, 100, 1),
    (5_000, 32, 10, 0), (3_000, 16, 50, 1), (2_000, 13, 300, 0),
]


@pytest.fixture(scope="module")
def B():
    from paper_1907_07410_amd import binding
    return binding


@pytest.mark.parametrize("n,k,K,prec", SHAPES)
def test_threshold_rank_is_the_poisson_quantile(B, n, k, K, prec):
    p = B.topk_plan(n, k, 4096, K, prec)
    need = p["need"]
    assert need == (K + max(16, K // 2) if prec == 1 else K)
    if need >= n or n <= 1024:
        assert p["samples"] == 0 and p["rank"] == 0
        return
    s, r = p["samples"], p["rank"]
    assert s == 1024
    lam = need * s / n
    if lam <= 50:
        # the smallest r with P(Poisson(lam) >= r) <= 1e-6
        assert stats.poisson.sf(r - 1, lam) <= 1e-6
        assert r == 1 or stats.poisson.sf(r - 2, lam) > 1e-6
    else:
        assert stats.poisson.sf(r - 1, lam) <= 1e-5


@pytest.mark.parametrize("n,k,K,prec", SHAPES)
def test_candidate_buffer_covers_the_sample_tail(B, n, k, K, prec):
    """The share of items at or above the r-th best of s sampled ones is
    Beta(r, s - r + 1); the buffer holds at least three times its mean plus
    slack, and overflows (which send a tile to the full selection) with
    probability at most about 1e-9 per user, unless the 8,192-key cap
    binds."""
    p = B.topk_plan(n, k, 4096, K, prec)
    if p["samples"] == 0:
        assert p["capacity"] >= n
        return
    s, r, cap = p["samples"], p["rank"], p["capacity"]
    assert cap % 64 == 0 and cap >= p["need"] + 64
    mean = r / (s + 1) * n
    assert cap >= min(8192, 3 * mean + 128)
    overflow = stats.beta.sf(cap / n, r, s - r + 1)
    if cap < 8192:
        assert overflow <= 2e-9, (r, cap, overflow)


def test_old_three_times_rule_overflowed_at_the_serving_tables():
    """Why the tail term exists: at 100,000 items and 150 BF16 candidates
    the rank is 11, and three times the mean (the buffer's former size)
    overflows for about one user in 1.7 million: about once in a serving
    stream of 2,000 requests (a million users scored)."""
    s, r, n = 1024, 11, 100_000
    old_cap = int(np.ceil((3 * r / (s + 1) * n + 128) / 64) * 64)
    assert old_cap == 3392
    assert 3e-7 < stats.beta.sf(old_cap / n, r, s - r + 1) < 1e-6


@pytest.mark.parametrize("n,k,K,prec", SHAPES)
@pytest.mark.parametrize("nu", [1, 17, 4096, 480_000])
def test_filter_splits(B, n, k, K, prec, nu):
    p = B.topk_plan(n, k, nu, K, prec)
    S, per = p["splits"], p["per_split"]
    assert per % 16 == 0 and per <= 65_536
    assert S * per >= n and (S - 1) * per < n
    # a multiple of 8 (one eighth of the item rows per XCD) while every
    # split keeps at least 256 items and the 16-bit offsets allow it
    if n >= 8 * 256 and S * 256 <= n and (n + 65519) // 65520 <= 8:
        assert S % 8 == 0 or S == -(-n // per)


def test_workspace_grows_with_users_and_matches_the_stated_limits(B):
    """bmf_topk_dev_noalloc takes requests whose workspace fits 64 MiB: about
    4,200 users at 27,000 items and k = 64, about 1,800 at 100,000 and
    k = 128 (K = 100, BF16 the larger)."""
    cap = 64 << 20

    def largest(n, k):
        lo, hi = 1, 1 << 16
        while lo < hi:
            mid = (lo + hi + 1) // 2
            need = max(B.topk_plan(n, k, mid, 100, prec)["workspace_bytes"] for prec in (0, 1))
            lo, hi = (mid, hi) if need <= cap else (lo, mid - 1)
        return lo

    a = largest(27_000, 64)
    b = largest(100_000, 128)
    assert 4_100 <= a <= 4_300, a
    assert 1_700 <= b <= 1_900, b
    w = [B.topk_plan(100_000, 128, nu, 100, 1)["workspace_bytes"] for nu in (16, 32, 1024)]
    assert w[0] < w[1] < w[2]


def test_bad_arguments_are_refused(B):
    for args in [(0, 64, 10, 10, 0), (1000, 0, 10, 10, 0), (1000, 300, 10, 10, 0), (1000, 64, 0, 10, 0),
                 (1000, 64, 10, 0, 0), (1000, 64, 10, 513, 0), (1000, 64, 10, 10, 3), (1000, 64, 10, 100, 1, 50)]:
        with pytest.raises(B.BmfError) as ex:
            B.topk_plan(*args)
        assert ex.value.status == B.BMF_E_INVAL
