"""Seeded synthetic rating data shaped like the paper's workloads.

This module only draws inputs: it holds none of the factorisation method's
arithmetic (no prediction, no update, no partition, no schedule).  Both the
HIP library's tests and the FP64 oracle's tests take their inputs from here.

Recipe (the paper evaluates on MovieLens/Jester, Section 5, which are not
available; these draws stand in for them):

* degrees: capped Zipf.  The rank-r entity gets weight r**-s; degrees are
  found by water-filling so that no degree exceeds the size of the opposite
  dimension and the degrees sum to the requested count.
* ids: ranks are mapped to ids through a seeded permutation, so that ids are
  uncorrelated with popularity.
* pairs: every user draws its d_u distinct items with probability
  proportional to the item weights (no duplicate (u, i) pairs).
* values: a planted low-rank model, offset + sum_f u_f v_f + Gaussian noise,
  with u, v ~ N(0, sigma_f^2), then rounded (integer stars or half stars) and
  clipped to the rating scale.
* split: a seeded random permutation, the first fraction is training data.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np


@dataclass
class Ratings:
    u: np.ndarray  # int32 user ids
    i: np.ndarray  # int32 item ids
    r: np.ndarray  # float32 ratings

    def __len__(self) -> int:
        return int(self.u.shape[0])

    def subset(self, idx: np.ndarray) -> "Ratings":
        return Ratings(self.u[idx].copy(), self.i[idx].copy(), self.r[idx].copy())


@dataclass
class Problem:
    m: int
    n: int
    train: Ratings
    test: Optional[Ratings]


# ----------------------------------------------------------------- degrees
def capped_zipf_degrees(count: int, total: int, s: float, cap: int) -> np.ndarray:
    """Integer degrees for ranks 1..count, proportional to rank**-s, each at
    most ``cap``, summing exactly to ``total`` (water-filling + largest
    remainder rounding)."""
    if total > count * cap:
        raise ValueError("total exceeds count*cap")
    w = np.arange(1, count + 1, dtype=np.float64) ** (-float(s))
    capped = np.zeros(count, dtype=bool)
    for _ in range(count + 1):
        rem = total - cap * capped.sum()
        scale = rem / w[~capped].sum()
        d = np.where(capped, float(cap), scale * w)
        over = d > cap
        if not (over & ~capped).any():
            break
        capped |= over
    d = np.minimum(d, float(cap))
    base = np.floor(d).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        frac = d - base
        frac[base >= cap] = -1.0
        order = np.argsort(-frac, kind="stable")
        base[order[:short]] += 1
    assert base.sum() == total and base.max() <= cap
    return base


def _weighted_distinct(rng: np.random.Generator, weights: np.ndarray, d: int) -> np.ndarray:
    """``d`` distinct indices drawn without replacement, probability
    proportional to ``weights`` (Gumbel top-d)."""
    n = weights.shape[0]
    if d >= n:
        return np.arange(n, dtype=np.int64)
    keys = np.log(weights) + rng.gumbel(size=n)
    return np.argpartition(-keys, d - 1)[:d].astype(np.int64)


def _workers(workers: Optional[int]) -> int:
    if workers is not None:
        return max(1, int(workers))
    try:
        import os
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except (AttributeError, OSError):
        return 1


def _light_pairs(rng: np.random.Generator, users: np.ndarray, deg: np.ndarray, cdf: np.ndarray,
                 n: int) -> np.ndarray:
    """Keys u * n + i of ``deg[q]`` distinct items for each user ``users[q]``,
    items drawn with probability given by ``cdf`` (redrawn until distinct)."""
    need = deg.copy()
    have = np.zeros(0, dtype=np.int64)
    for _ in range(200):
        todo = need > 0
        if not todo.any():
            return have
        uu = np.repeat(users[todo], need[todo])
        draws = np.minimum(np.searchsorted(cdf, rng.random(uu.shape[0]), side="right"), n - 1)
        have = np.unique(np.concatenate([have, uu * np.int64(n) + draws]))
        cnt = np.searchsorted(have, (users + 1) * np.int64(n)) - np.searchsorted(have, users * np.int64(n))
        need = deg - cnt
    raise RuntimeError("pair sampler did not converge")


def sample_pairs_zipf(m: int, n: int, nnz: int, s_user: float, s_item: float,
                      rng: np.random.Generator, workers: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Distinct (u, i) pairs with capped-Zipf user degrees and item
    popularity, returned sorted by a random key (not by user).  Users with a
    quarter or more of all items draw theirs by Gumbel top-d; the others are
    drawn in chunks of consecutive user ids, each chunk from its own child
    stream of ``rng`` (so the result does not depend on ``workers``)."""
    du_rank = capped_zipf_degrees(m, nnz, s_user, n)
    wi_rank = capped_zipf_degrees(n, nnz, s_item, m).astype(np.float64) + 1e-3
    uperm = rng.permutation(m)
    iperm = rng.permutation(n)
    deg = np.empty(m, dtype=np.int64)
    deg[uperm] = du_rank
    w = np.empty(n, dtype=np.float64)
    w[iperm] = wi_rank
    heavy = deg >= max(1, n // 4)
    keys = []
    for u in np.nonzero(heavy)[0]:
        items = _weighted_distinct(rng, w, int(deg[u]))
        keys.append(u * np.int64(n) + items)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    light_users = np.nonzero(~heavy)[0]
    # chunks of about 2M ratings of consecutive users
    csum = np.cumsum(deg[light_users])
    nchunk = max(1, int(csum[-1] // (1 << 21)) + 1) if light_users.size else 0
    bounds = np.searchsorted(csum, np.linspace(0, csum[-1] if light_users.size else 0, nchunk + 1)[1:-1])
    parts = np.split(np.arange(light_users.size), bounds) if nchunk else []
    streams = rng.spawn(len(parts)) if parts else []

    def one(q: int) -> np.ndarray:
        idx = parts[q]
        return _light_pairs(streams[q], light_users[idx], deg[light_users[idx]], cdf, n)

    nw = _workers(workers)
    if nw > 1 and len(parts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=nw) as ex:
            keys.extend(ex.map(one, range(len(parts))))
    else:
        keys.extend(one(q) for q in range(len(parts)))
    allk = np.concatenate(keys) if keys else np.zeros(0, dtype=np.int64)
    if allk.shape[0] != nnz:
        raise RuntimeError("pair sampler drew the wrong count")
    allk = allk[rng.permutation(nnz)]
    return (allk // n).astype(np.int32), (allk % n).astype(np.int32)


def sample_pairs_uniform(m: int, n: int, nnz: int, rng: np.random.Generator):
    cells = rng.choice(m * n, size=nnz, replace=False)
    return (cells // n).astype(np.int32), (cells % n).astype(np.int32)


# ----------------------------------------------------------------- values
def planted_values(u: np.ndarray, i: np.ndarray, m: int, n: int, rank: int,
                   sigma_f: float, noise: float, offset: float, rounding: str,
                   rng: np.random.Generator, chunk: int = 1 << 21,
                   workers: Optional[int] = None) -> np.ndarray:
    """offset + <U_u, V_i> + N(0, noise^2), rounded and clipped.

    rounding: "int" -> clip(round(y), 1, 5); "half" -> clip(round(2y)/2,
    0.5, 5); "none" -> y unchanged.  numpy rounds half to even.  The noise of
    each chunk of ratings comes from its own child stream of ``rng`` (so the
    result does not depend on ``workers``)."""
    if rounding not in ("int", "half", "none"):
        raise ValueError(rounding)
    U = rng.normal(0.0, sigma_f, size=(m, rank)).astype(np.float32)
    V = rng.normal(0.0, sigma_f, size=(n, rank)).astype(np.float32)
    out = np.empty(u.shape[0], dtype=np.float32)
    starts = list(range(0, u.shape[0], chunk))
    streams = rng.spawn(len(starts)) if starts else []

    def one(q: int) -> None:
        s = starts[q]
        e = min(s + chunk, u.shape[0])
        y = np.einsum("ij,ij->i", U[u[s:e]], V[i[s:e]], dtype=np.float64)
        y += offset
        if noise > 0:
            y += streams[q].normal(0.0, noise, size=e - s)
        if rounding == "int":
            y = np.clip(np.round(y), 1.0, 5.0)
        elif rounding == "half":
            y = np.clip(np.round(2.0 * y) / 2.0, 0.5, 5.0)
        out[s:e] = y

    nw = _workers(workers)
    if nw > 1 and len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=nw) as ex:
            list(ex.map(one, range(len(starts))))
    else:
        for q in range(len(starts)):
            one(q)
    return out


def split(rat: Ratings, train_frac: float, rng: np.random.Generator):
    """Seeded random split: the first ``train_frac`` of a random permutation
    is training data; both parts keep the input order."""
    perm = rng.permutation(len(rat))
    cut = int(round(train_frac * len(rat)))
    train = np.zeros(len(rat), dtype=bool)
    train[perm[:cut]] = True
    return rat.subset(np.flatnonzero(train)), rat.subset(np.flatnonzero(~train))


# ----------------------------------------------------------------- helpers
def random_coo(m: int, n: int, nnz: int, seed: int, dup: bool = False,
               lo: float = 1.0, hi: float = 5.0) -> Ratings:
    """Small unstructured COO for edge-case tests (duplicates allowed when
    ``dup``)."""
    rng = np.random.default_rng(seed)
    if dup:
        u = rng.integers(0, m, size=nnz).astype(np.int32)
        i = rng.integers(0, n, size=nnz).astype(np.int32)
    else:
        u, i = sample_pairs_uniform(m, n, nnz, rng)
    r = rng.uniform(lo, hi, size=nnz).astype(np.float32)
    return Ratings(u, i, r)


def serving_factors(m: int, n: int, k: int, seed: int, sigma: float = 0.3,
                    correlated: bool = False):
    """Factor tables for the serving workload: i.i.d. N(0, sigma^2) entries
    (or, when ``correlated``, a decaying spectrum that makes near ties more
    frequent), biases N(0, sigma^2), global mean 3.5."""
    rng = np.random.default_rng(seed)
    P = rng.normal(0.0, sigma, size=(m, k)).astype(np.float32)
    Q = rng.normal(0.0, sigma, size=(n, k)).astype(np.float32)
    if correlated:
        scale = (1.0 / np.sqrt(1.0 + np.arange(k))).astype(np.float32)
        P *= scale
        Q *= scale
    bu = rng.normal(0.0, sigma, size=m).astype(np.float32)
    bi = rng.normal(0.0, sigma, size=n).astype(np.float32)
    return P, Q, bu, bi, 3.5
