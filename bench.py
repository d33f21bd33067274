"""Benchmark: stratified block-SGD training of biased MF on the mid-scale
synthetic workload (138,000 users x 27,000 items, 20M Zipf(1.1) ratings,
half stars, 90/10 split, k=64, 64 x 64 blocks, lr 0.005, reg 0.05).

One step = one iteration of the paper's Algorithm 1: one epoch over every
training rating (b strata of b concurrent blocks) followed by the test RMSE
(the quantity the stopping rule watches).  value = training rating updates
per second over the timed steps, inputs resident in HBM.

Also reported: the SGD kernel's achieved algorithmic HBM bandwidth against
the MI355X peak, the FP64 oracle timed on the host cores on one epoch, the
one-epoch parity of the GPU factors against that oracle epoch, and top-100
throughput for a batch of users in FP32 and BF16 scoring.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(u, i, m, n, b, k):
    """Bytes one epoch must move: every rating record once (8 B), plus, per
    block, each distinct user row and item row (k factors + bias, FP32) read
    once and written once."""
    rb, cb = -(-m // b), -(-n // b)
    blk = (u.astype(np.int64) // rb) * b + (i.astype(np.int64) // cb)
    users = np.unique(blk * m + u).shape[0]
    items = np.unique(blk * n + i).shape[0]
    return u.shape[0] * 8 + (users + items) * (k + 1) * 4 * 2, users, items


def critical_path(u, i, m, n, b, order_mode=0):
    """Sum over strata of the largest block's rating count (the dependent
    update chain with one wavefront per block)."""
    rb, cb = -(-m // b), -(-n // b)
    blk = (u.astype(np.int64) // rb) * b + (i.astype(np.int64) // cb)
    cnt = np.bincount(blk, minlength=b * b).reshape(b, b)
    tot = 0
    for s in range(b):
        tot += max(cnt[(j + s) % b, j] for j in range(b))
    return int(tot), int(cnt.max()), float(cnt.mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--topk-users", type=int, default=4096)
    ap.add_argument("--sgd-kernel", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (sharding is described in "
              "DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.warmup < 1:
        args.warmup = 1

    import torch
    from paper_1907_07410_amd import binding, configs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    cfg = configs.MID
    t0 = time.time()
    prob = cfg.generate(args.seed)
    tr, te = prob.train, prob.test
    log(f"generated {len(tr)} train / {len(te)} test ratings in {time.time() - t0:.1f}s")
    abytes, nu_blk, ni_blk = algorithmic_bytes(tr.u, tr.i, prob.m, prob.n, cfg.b, cfg.k)
    cp, maxblk, meanblk = critical_path(tr.u, tr.i, prob.m, prob.n, cfg.b)
    log(f"algorithmic bytes/epoch {abytes / 1e9:.3f} GB; critical path {cp} ratings")

    G = binding.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0,
                      order_seed=args.seed + 2000, sgd_kernel=args.sgd_kernel)
    t0 = time.time()
    G.load_ratings(tr.u, tr.i, tr.r)
    load_s = time.time() - t0
    log(f"load + partition {load_s:.2f}s")

    # first warm-up epoch, then compare with the oracle's first epoch
    G.epoch(cfg.lr, cfg.reg)
    G.synchronize()
    parity = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        threads = max(1, min(threads, 64))
        O = oracle.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0)
        O.load(tr.u, tr.i, tr.r)
        t0 = time.time()
        O.epoch(cfg.lr, cfg.reg, threads=threads)
        cpu_s = time.time() - t0
        cpu = {"value": len(tr) / cpu_s, "unit": "rating updates/s", "cores": threads, "kind": "oracle",
               "sample": f"one full epoch of the mid-scale workload ({len(tr)} updates, FP64, "
                         f"{threads} threads over each stratum's blocks)"}
        P, Q, bu, bi, mu = G.get_factors()
        parity = float(max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(),
                           np.abs(bi - O.bi).max()))
        log(f"oracle epoch {cpu_s:.1f}s on {threads} threads; 1-epoch max abs diff {parity:.3g}")
        del O
    for _ in range(args.warmup - 1):
        G.epoch(cfg.lr, cfg.reg)
    G.synchronize()
    G.sgd_timing(reset=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rmse = None
    for _ in range(args.steps):
        G.epoch(cfg.lr, cfg.reg)
        rmse = G.rmse(te.u, te.i, te.r)
    G.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sgd_ms, launches = G.sgd_timing(reset=True)
    value = len(tr) * args.steps / el
    per_launch_ms = sgd_ms / max(1, launches)
    achieved = (abytes / cfg.b) / (per_launch_ms / 1e3) / 1e9
    log(f"{args.steps} steps in {el:.3f}s; sgd kernels {sgd_ms:.2f} ms over {launches} launches; test rmse {rmse:.4f}")

    # top-100 for a batch of users, FP32 and BF16 scoring
    topk = {}
    if args.topk_users > 0:
        rng = np.random.default_rng(7)
        users = rng.integers(0, prob.m, args.topk_users).astype(np.int32)
        res = {}
        for name, fn in (("fp32", lambda: G.topk(users, 100)), ("bf16", lambda: G.topk_bf16(users, 100))):
            fn()
            t0 = time.perf_counter()
            out = fn()
            dt = time.perf_counter() - t0
            res[name] = out
            topk[name + "_users_per_s"] = len(users) / dt
            topk[name + "_ms"] = dt * 1e3
        recall = float(np.mean([len(set(a) & set(b)) / 100 for a, b in zip(res["fp32"][0], res["bf16"][0])]))
        topk["recall_at_100_bf16_vs_fp32"] = recall
        topk["users"] = len(users)
        topk["items"] = prob.n

    line = {
        "metric": "rating updates/s at matched RMSE; top-100 req/s + p99 latency (BF16 vs FP32)",
        "value": value,
        "unit": "rating updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mid-scale: 138000 users x 27000 items, 20M Zipf(1.1) ratings (18M train), "
                               "k=64, 64x64 blocks, lr 0.005, reg 0.05",
                   "m": prob.m, "n": prob.n, "n_train": len(tr), "k": cfg.k, "b": cfg.b},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sgd stratum kernel", "algorithmic_bytes_per_launch": abytes / cfg.b,
                     "avg_launch_ms": per_launch_ms},
        "cpu_baseline": cpu,
        "rmse_test": rmse,
        "parity_1epoch_max_abs": parity,
        "critical_path_ratings_per_epoch": cp,
        "load_s": load_s,
        "topk": topk,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
