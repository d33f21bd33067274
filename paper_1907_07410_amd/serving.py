"""Request streams for the serving engine.

A request is a top-K query for a batch of existing users (batch size
log-uniform on [1, 4096], user ids drawn by Zipf popularity) or a new-user
fold-in (5-500 (item, rating) pairs, log-uniform, items by Zipf
popularity, ratings from a planted user vector through the model's item
factors, rounded and clipped to 1-5).  Arrivals are Poisson.  This module
only draws requests and drives a binding.Server; latency is measured by the
server (submit to completion).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np


@dataclass
class Req:
    t: float                      # arrival time (s) from the start of the run
    kind: str                     # "topk" or "foldin"
    users: Optional[np.ndarray] = None
    items: Optional[np.ndarray] = None
    ratings: Optional[np.ndarray] = None


def zipf_ids(rng, count, size, s=1.1, perm=None):
    """Ids in [0, count) with probability proportional to rank**-s (ranks
    mapped to ids through `perm`)."""
    w = np.arange(1, count + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    ranks = np.minimum(np.searchsorted(cdf, rng.random(size), side="right"), count - 1)
    return ranks if perm is None else perm[ranks]


def make_stream(rng, n_req, rate, m, n, Q, bi, mu, topk_frac=0.9, batch_range=(1, 4096), foldin_range=(5, 500),
                sigma=0.3) -> List[Req]:
    uperm = rng.permutation(m)
    iperm = rng.permutation(n)
    t = np.cumsum(rng.exponential(1.0 / rate, n_req)) if rate > 0 else np.zeros(n_req)
    out = []
    k = Q.shape[1]
    for q in range(n_req):
        if rng.random() < topk_frac:
            bs = int(np.exp(rng.uniform(np.log(batch_range[0]), np.log(batch_range[1] + 1))))
            bs = max(batch_range[0], min(batch_range[1], bs))
            out.append(Req(float(t[q]), "topk", users=zipf_ids(rng, m, bs, perm=uperm).astype(np.int32)))
        else:
            nr = int(np.exp(rng.uniform(np.log(foldin_range[0]), np.log(foldin_range[1] + 1))))
            nr = max(foldin_range[0], min(foldin_range[1], nr))
            items = np.unique(zipf_ids(rng, n, nr * 2, perm=iperm))[:nr]
            rng.shuffle(items)
            p_true = rng.normal(0, sigma, k)
            y = mu + bi[items] + Q[items] @ p_true + rng.normal(0, 0.5, items.shape[0])
            out.append(Req(float(t[q]), "foldin", items=items.astype(np.int32),
                           ratings=np.clip(np.round(y), 1, 5).astype(np.float32)))
    return out


def run(server, reqs: List[Req], K=100, precision=1) -> dict:
    """Submit `reqs` at their arrival times (open loop), wait for all, and
    return the server's statistics plus the achieved request rate."""
    server.stats(reset=True)
    t0 = time.perf_counter()
    ids = []
    for r in reqs:
        while time.perf_counter() - t0 < r.t:
            pass
        if r.kind == "topk":
            ids.append(server.submit_topk(r.users, K, precision))
        else:
            ids.append(server.submit_foldin(r.items, r.ratings, K, precision))
    server.drain()
    elapsed = time.perf_counter() - t0
    for rid in ids:
        server.poll(rid, wait=True)
    st = server.stats()
    st["elapsed_s"] = elapsed
    st["req_per_s"] = len(reqs) / elapsed
    st["offered_req_per_s"] = len(reqs) / max(reqs[-1].t, 1e-9) if reqs and reqs[-1].t > 0 else None
    return st
