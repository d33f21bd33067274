"""Benchmark: stratified block-SGD training of biased MF (the paper's
Algorithm 1 with Algorithm 2 per block) on one MI355X.

Headline workload (the largest single-problem configuration): 480,000 users
x 17,800 items, 100M Zipf(1.0) integer ratings from a planted rank-64 model,
90/10 split (90M training ratings), k=128, 128 x 128 blocks, lr 0.005,
reg 0.05.  One step = one iteration of Algorithm 1: one epoch over every
training rating (b strata of b concurrent blocks) followed by the test RMSE
(what the stopping rule watches).  value = training rating updates per
second over the timed steps, inputs resident in HBM.  The run's RMSE after
the configuration's 20 epochs is compared with the FP64 oracle's
("matched RMSE").

Also reported: the SGD stratum kernel against the HBM roof (algorithmic
bytes per launch over the HIP-event launch time) and against the
dependency-chain bound it actually runs into (critical plan steps per epoch
times the measured time of one dependent step), the FP64 oracle timed on the
host cores, top-100 for every user in FP32 and BF16 scoring, and further
legs: the mid workload (138,000 x 27,000, 18M training ratings, k=64,
64 x 64 blocks), serving, batched training, the paper's protocol,
incremental data and out-of-core training.
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
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}  # MI355X dense matrix peaks

# HBM bytes per launch of the SGD stratum kernel per workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE), each scaled by the factor
# that makes the same counter read a plain copy kernel's known bytes; valid
# for the kernel sources with this sha1 and reported as null once they
# change.
SGD_TRAFFIC = {"large": {"sources_sha1": "cf312bb15e1872c0a1b5821fe1b23c33324da22a",
                         "fetch_bytes": 61719.5 * 1024 * 2.0, "write_bytes": 111948.0 * 1024 * 1.0}}
SGD_SOURCES = ["paper_1907_07410_amd/csrc/sgd.hip", "paper_1907_07410_amd/csrc/plan.hip",
               "paper_1907_07410_amd/csrc/plan.h", "paper_1907_07410_amd/csrc/wave.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sources_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in SGD_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    t = SGD_TRAFFIC.get(workload)
    if t is None or t["sources_sha1"] != sources_sha1():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def algorithmic_bytes(u, i, m, n, b, k):
    """Bytes one epoch must move: every rating record once (8 B), plus, per
    block, each distinct user row and item row (k factors + bias, FP32) read
    once and written once.  A user's block row is fixed by the user, so the
    distinct (block, user) pairs are the distinct (user, block column)
    pairs; likewise for items."""
    rb, cb = -(-m // b), -(-n // b)
    seen = np.zeros(m * b, dtype=bool)
    seen[u.astype(np.int64) * b + i // cb] = True
    users = int(np.count_nonzero(seen))
    del seen
    seen = np.zeros(n * b, dtype=bool)
    seen[i.astype(np.int64) * b + u // rb] = True
    items = int(np.count_nonzero(seen))
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


def tables_recall(G, P, Q, bu, bi, mu, K, users, n64=32):
    """Top-K of ``users`` in FP32 and in BF16 with FP32 rescoring: BF16
    recall@K against FP32, and both against FP64 scores of the same factors
    on the first ``n64`` users (recall and the largest score error)."""
    f_it, f_sc = G.topk(users, K)
    b_it, b_sc = G.topk_bf16(users, K)
    out = {"users": int(len(users)),
           "recall_bf16_vs_fp32": float(np.mean([len(set(a) & set(b)) / K for a, b in zip(f_it, b_it)]))}
    Qd, bid = Q.astype(np.float64), bi.astype(np.float64)
    rec = {"fp32": [], "bf16": []}
    err = {"fp32": 0.0, "bf16": 0.0}
    for row in range(min(n64, len(users))):
        uu = users[row]
        s64 = mu + float(bu[uu]) + bid + Qd @ P[uu].astype(np.float64)
        best = set(np.argsort(-s64, kind="stable")[:K].tolist())
        for name, its, scs in (("fp32", f_it[row], f_sc[row]), ("bf16", b_it[row], b_sc[row])):
            rec[name].append(len(best & set(its.tolist())) / K)
            err[name] = max(err[name], float(np.abs(scs.astype(np.float64) - s64[its]).max()))
    for name in ("fp32", "bf16"):
        out[f"recall_{name}_vs_fp64"] = float(np.mean(rec[name]))
        out[f"max_score_error_{name}_vs_fp64"] = err[name]
    out["fp64_users"] = min(n64, len(users))
    return out


# Poisson loads as fractions of each server's own saturated rate
SERVING_LOADS = (0.1, 0.2, 0.3, 0.4, 0.5, 0.7, 0.9, 1.2)


def serving_leg(binding, args):
    """Top-100 serving on the 1M-user x 100k-item, k=128 factor tables:
    the continuous-batching server scoring in BF16 (FP32 rescoring), the same
    server scoring in FP32, and an FP32 server that runs one request at a
    time.  Each runs the same request stream submitted at once (saturated
    throughput), then Poisson streams of twice as many requests at 10% to
    120% of its own saturated rate (latency at load); req/s at a stated p99
    compares the three."""
    from paper_1907_07410_amd import configs, serving, synth
    sc = configs.SERVING
    t0 = time.time()
    P, Q, bu, bi, mu = synth.serving_factors(sc.m, sc.n, sc.k, seed=args.seed + 3)
    G = binding.Model(sc.m, sc.n, sc.k, 1)
    G.set_factors(P, Q, bu, bi, mu)
    log(f"serving tables {sc.m} x {sc.n} x {sc.k} ready in {time.time() - t0:.1f}s")
    # recall of BF16 scoring on these tables and on tables with a decaying
    # spectrum (scale 1/sqrt(1+f) on factor f), the harder case for it
    rrng = np.random.default_rng(args.seed + 14)
    recall = {"iid": tables_recall(G, P, Q, bu, bi, mu, sc.K, rrng.integers(0, sc.m, 4096).astype(np.int32))}
    del P, bu
    P2, Q2, bu2, bi2, mu2 = synth.serving_factors(sc.m, sc.n, sc.k, seed=args.seed + 4, correlated=True)
    G2 = binding.Model(sc.m, sc.n, sc.k, 1)
    G2.set_factors(P2, Q2, bu2, bi2, mu2)
    recall["decaying_spectrum"] = tables_recall(G2, P2, Q2, bu2, bi2, mu2, sc.K,
                                                rrng.integers(0, sc.m, 4096).astype(np.int32))
    G2.close()
    del P2, Q2, bu2, bi2, G2
    log("serving tables recall@100 BF16 vs FP32: " + ", ".join(
        f"{name} {v['recall_bf16_vs_fp32']:.6f} (vs FP64 {v['recall_bf16_vs_fp64']:.4f})" for name, v in recall.items()))
    rng = np.random.default_rng(args.seed + 11)
    n = args.serving_requests
    reqs = serving.make_stream(rng, n, 0, sc.m, sc.n, Q, bi, mu, topk_frac=sc.topk_frac,
                               batch_range=sc.batch_range, foldin_range=sc.foldin_range)
    warm = serving.make_stream(rng, 8, 0, sc.m, sc.n, Q, bi, mu, topk_frac=sc.topk_frac,
                               batch_range=sc.batch_range, foldin_range=sc.foldin_range)
    out = {"tables": f"{sc.m} x {sc.n}, k={sc.k}", "K": sc.K, "requests": n, "recall": recall,
           "mix": f"{int(sc.topk_frac * 100)}% top-{sc.K} for log-uniform {sc.batch_range} users, "
                  f"rest fold-in of log-uniform {sc.foldin_range} ratings"}
    users = sum(len(r.users) for r in reqs if r.kind == "topk")
    # three servers on the same streams: BF16 scoring with continuous
    # batching, FP32 scoring with the same batching (what BF16 adds on its
    # own), and FP32 one request at a time (the unbatched baseline)
    for name, kw, prec in (("bf16_continuous_batching", dict(), 1),
                           ("fp32_continuous_batching", dict(), 0),
                           ("fp32_one_request_per_batch", dict(max_batches=1, max_requests_per_batch=1), 0)):
        S = binding.Server(G, mem_budget_bytes=4 << 30, foldin_passes=sc.foldin_passes, foldin_lr=sc.lr,
                           foldin_reg=sc.reg, **kw)
        serving.run(S, warm, K=sc.K, precision=prec)
        st = serving.run(S, reqs, K=sc.K, precision=prec)
        sat = st["req_per_s"]
        # one unmeasured Poisson stream first: the first open-loop stream
        # after the saturated run has shown a single stall of about 10 ms in
        # the runtime (a launch call blocked while every batch in flight
        # waited), and later streams have not
        prng = np.random.default_rng(args.seed + 13)
        serving.run(S, serving.make_stream(prng, n, 0.5 * sat, sc.m, sc.n, Q, bi, mu, topk_frac=sc.topk_frac,
                                           batch_range=sc.batch_range, foldin_range=sc.foldin_range),
                    K=sc.K, precision=prec)
        sweep = []
        for frac in SERVING_LOADS:
            prng = np.random.default_rng(args.seed + 12)
            # twice the saturated stream's length: the p99 is then the 20th
            # slowest request, less at the mercy of one slow burst
            preqs = serving.make_stream(prng, 2 * n, frac * sat, sc.m, sc.n, Q, bi, mu, topk_frac=sc.topk_frac,
                                        batch_range=sc.batch_range, foldin_range=sc.foldin_range)
            stp = serving.run(S, preqs, K=sc.K, precision=prec)
            sweep.append({"load": frac, "offered_req_per_s": frac * sat, "achieved_req_per_s": stp["req_per_s"],
                          "p50_ms": stp["p50_ms"], "p99_ms": stp["p99_ms"]})
        st2 = sweep[SERVING_LOADS.index(0.5)]
        out[name] = {"saturated_req_per_s": sat, "saturated_users_per_s": users / st["elapsed_s"],
                     "saturated_p50_ms": st["p50_ms"], "saturated_p99_ms": st["p99_ms"],
                     "batches": st["batches"], "poisson_offered_req_per_s": 0.5 * sat,
                     "poisson_achieved_req_per_s": st2["achieved_req_per_s"], "poisson_p50_ms": st2["p50_ms"],
                     "poisson_p99_ms": st2["p99_ms"], "poisson_sweep": sweep}
        log(f"serving {name}: {sat:.1f} req/s saturated (p99 {st['p99_ms']:.1f} ms); Poisson p99 at "
            + "/".join(f"{int(round(f * 100))}" for f in SERVING_LOADS) + "%: "
            + " / ".join(f"{x['p99_ms']:.2f}" for x in sweep) + " ms")
        S.close()
    # the largest achieved rate among each server's load points whose p99
    # stays within a stated latency objective
    slo = {}
    for slo_ms in (2.0, 5.0, 10.0):
        row = {}
        for name in ("bf16_continuous_batching", "fp32_continuous_batching", "fp32_one_request_per_batch"):
            ok = [x["achieved_req_per_s"] for x in out[name]["poisson_sweep"] if x["p99_ms"] <= slo_ms]
            row[name] = max(ok) if ok else None
        slo[f"p99_le_{slo_ms:g}ms"] = row
    out["req_per_s_at_p99_slo"] = slo
    log("serving req/s at p99 <= 5 ms: " + ", ".join(f"{k2} {v}" for k2, v in slo["p99_le_5ms"].items()))
    # fold-in latency alone (host call: upload, 10 passes, download), k = 128
    fold = {}
    frng = np.random.default_rng(args.seed + 13)
    for nr in (5, 50, 500):
        items = frng.choice(sc.n, nr, replace=False).astype(np.int32)
        r = frng.integers(1, 6, nr).astype(np.float32)
        G.foldin(items, r, sc.foldin_passes, sc.lr, sc.reg)
        lat = []
        for _ in range(20):
            t0 = time.perf_counter()
            G.foldin(items, r, sc.foldin_passes, sc.lr, sc.reg)
            lat.append((time.perf_counter() - t0) * 1e3)
        fold[str(nr)] = {"median_ms": float(np.median(lat)), "max_ms": float(np.max(lat))}
    out["foldin_latency_k128_10_passes"] = fold
    log("fold-in latency (5 / 50 / 500 ratings): " + " / ".join(f"{v['median_ms']:.3f}" for v in fold.values()) + " ms")
    del G
    return out


def batched_leg(binding, args, torch):
    """64 independent problems of uneven size (users U[10k, 200k], items
    U[2k, 50k], density 0.1-1%, Zipf(1.1) degrees, k=32) scaled linearly in
    users and items by --batched-scale, trained together with autotuned block
    grids; 10 timed epochs after one warm-up epoch.  Also times one epoch of
    every problem run alone (one after another) for comparison."""
    from paper_1907_07410_amd import configs
    bc = configs.BATCHED
    t0 = time.time()
    done = []

    def progress(p):
        done.append(p)
        if len(done) % 16 == 0:
            log(f"batched: {len(done)} of {bc.nprob} problems generated ({time.time() - t0:.0f}s)")

    probs = bc.generate(args.seed, args.batched_scale, workers=min(16, os.cpu_count() or 1), progress=progress)
    nnz = [len(p.train) for p in probs]
    log(f"batched: {len(probs)} problems, {sum(nnz)} ratings generated in {time.time() - t0:.1f}s")
    bt = binding.Batch([(p.m, p.n) for p in probs], bc.k, seed=args.seed + 1000)
    t0 = time.time()
    for q, p in enumerate(probs):
        bt.load(q, p.train.u, p.train.i, p.train.r)
    log(f"batched: loaded in {time.time() - t0:.1f}s")
    t0 = time.time()
    bt.tune()
    tune_s = time.time() - t0
    log(f"batched: grids and waves chosen in {tune_s:.1f}s")
    grids = [bt.info(q)[0] for q in range(len(probs))]
    waves = bt.info(0)[1]
    bt.epochs(1, bc.lr, bc.reg)
    bt.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.epochs(bc.epochs, bc.lr, bc.reg)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, launches = bt.timing(reset=True)
    alone_ms = 0.0
    for q in range(len(probs)):
        G = bt.problem(q)
        G.sgd_timing(reset=True)
        G.epoch(bc.lr, bc.reg)
        G.synchronize()
        alone_ms += G.sgd_timing(reset=True)[0]
    # Properties that hold at any size: every problem's training RMSE is
    # finite, and sampled problems (the largest, the smallest, two more)
    # equal the same problem trained alone on its grid for as many epochs
    # (1 + epochs batched, then the one alone epoch above), bit for bit.
    train_rmse = [bt.problem(q).rmse() for q in range(len(probs))]
    picks = sorted({int(np.argmax(nnz)), int(np.argmin(nnz)), 0, len(probs) // 2})
    same = {}
    for q in picks:
        p = probs[q]
        G = binding.Model(p.m, p.n, bc.k, bt.info(q)[0], seed=args.seed + 1000)
        G.load_ratings(p.train.u, p.train.i, p.train.r)
        for _ in range(bc.epochs + 2):
            G.epoch(bc.lr, bc.reg)
        got, want = bt.problem(q).get_factors(), G.get_factors()
        same[str(q)] = all(np.array_equal(x.view(np.uint32), y.view(np.uint32)) for x, y in zip(got[:4], want[:4]))
        G.close()
    log(f"batched: train RMSE {min(train_rmse):.4f}-{max(train_rmse):.4f}; alone bit-identical {same}")
    # algorithmic bytes of an epoch of every problem on its grid (as for one
    # problem: records once, each distinct row of each block in and out)
    abytes = sum(algorithmic_bytes(p.train.u, p.train.i, p.m, p.n, g, bc.k)[0] for p, g in zip(probs, grids))
    out = {"problems": len(probs), "scale": args.batched_scale, "ratings": int(sum(nnz)), "k": bc.k,
           "epochs": bc.epochs, "updates_per_s": sum(nnz) * bc.epochs / el, "epoch_ms": el * 1e3 / bc.epochs,
           "kernel_ms_per_epoch": ms / bc.epochs, "launches_per_epoch": launches / bc.epochs,
           "alone_sequential_epoch_ms": alone_ms, "speedup_vs_alone": alone_ms / (ms / bc.epochs),
           "tune_s": tune_s, "waves": waves, "grids": {str(b): grids.count(b) for b in sorted(set(grids))},
           "train_rmse_range": [min(train_rmse), max(train_rmse)],
           "alone_bit_identical": same,
           "algorithmic_bytes_per_epoch": abytes,
           "achieved_GBps": abytes / (ms / bc.epochs / 1e3) / 1e9,
           "frac_of_hbm_peak": abytes / (ms / bc.epochs / 1e3) / 1e9 / HBM_PEAK_GBS}
    log(f"batched: {out['updates_per_s'] / 1e6:.0f}M updates/s, epoch {out['epoch_ms']:.2f} ms "
        f"(alone one after another {alone_ms:.2f} ms), grids {out['grids']}, waves {waves}, tune {tune_s:.1f}s, "
        f"{out['achieved_GBps']:.0f} GB/s algorithmic")
    bt.close()
    return out


def paper_leg(binding, args):
    """Section 5's protocol on the MovieLens-1M-shaped workload (6,040 x
    3,883, 800,167 training ratings, k = 13, the paper's named pairs, early
    termination at delta = 1e-4), over three data seeds as Table 1 does:
    seconds per iteration and test RMSE at the grids of Table 1's rows, 8 x 8
    (BCSVD) and 3072 x 3072 (BGSVD) fitted to the stopping rule, 1 x 1 (plain
    SVD, one block on the reference kernel) timed over two epochs; the
    oracle's 8 x 8 fit and 1 x 1 epochs on the host beside them.  The
    paper's own Table 1 figures (other data, other machines) are attached as
    context."""
    from paper_1907_07410_amd import configs
    c = configs.PAPER_ML1M
    seeds = (args.seed, args.seed + 1, args.seed + 2)
    runs = {"gpu_b8": [], "gpu_b3072": [], "gpu_b3072_graph": [], "gpu_b1": [], "oracle_b8": [], "oracle_b1": []}
    threads = max(1, min(len(os.sched_getaffinity(0)), 8))
    for seed in seeds:
        prob = c.generate(seed)
        tr, te = prob.train, prob.test
        for b, graph in ((8, False), (3072, False), (3072, True)):
            name = f"gpu_b{b}" + ("_graph" if graph else "")
            G = binding.Model(prob.m, prob.n, c.k, b, seed=seed + 1000, order_mode=0)
            if graph:  # the epoch's 3072 launches replayed from a HIP graph
                G.set_option(binding.OPT_EPOCH_GRAPH, 1)
            t0 = time.perf_counter()
            G.load_ratings(tr.u, tr.i, tr.r)
            load_s = time.perf_counter() - t0
            G.epoch_hp([0.0] * 8)  # warm-up launch: zero rates leave the factors as they are
            G.synchronize()
            t0 = time.perf_counter()
            e, r = G.fit(configs.PAPER_HP, 1000, configs.PAPER_DELTA)
            el = time.perf_counter() - t0
            runs[name].append({"seed": seed, "epochs": e, "s_per_iter": el / e, "train_rmse": r,
                               "test_rmse": G.rmse(te.u, te.i, te.r), "load_s": load_s})
            log(f"paper protocol seed {seed} {name}: {e} epochs, {el / e * 1e3:.2f} ms/iter, test rmse "
                f"{runs[name][-1]['test_rmse']:.4f}, load {load_s:.2f}s")
            del G
        G = binding.Model(prob.m, prob.n, c.k, 1, seed=seed + 1000, order_mode=0)
        G.load_ratings(tr.u, tr.i, tr.r)
        G.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            G.epoch_hp(configs.PAPER_HP)
        G.synchronize()
        runs["gpu_b1"].append({"seed": seed, "epochs_timed": 2, "s_per_iter": (time.perf_counter() - t0) / 2})
        del G
        if args.no_cpu_baseline:
            continue
        import oracle
        O = oracle.Model(prob.m, prob.n, c.k, 8, seed=seed + 1000, order_mode=0)
        O.load(tr.u, tr.i, tr.r)
        t0 = time.perf_counter()
        e, r = O.fit(configs.PAPER_HP, 1000, configs.PAPER_DELTA, threads=threads)
        el = time.perf_counter() - t0
        runs["oracle_b8"].append({"seed": seed, "epochs": e, "s_per_iter": el / e, "train_rmse": r,
                                  "test_rmse": O.rmse(te.u, te.i, te.r), "threads": threads})
        O = oracle.Model(prob.m, prob.n, c.k, 1, seed=seed + 1000, order_mode=0)
        O.load(tr.u, tr.i, tr.r)
        t0 = time.perf_counter()
        for _ in range(2):
            O.epoch(hp=configs.PAPER_HP)
        runs["oracle_b1"].append({"seed": seed, "epochs_timed": 2, "s_per_iter": (time.perf_counter() - t0) / 2,
                                  "threads": 1})
        log(f"paper protocol seed {seed} oracle b=8: {e} epochs, {el / e * 1e3:.1f} ms/iter on {threads} threads, "
            f"test rmse {runs['oracle_b8'][-1]['test_rmse']:.4f}; b=1 "
            f"{runs['oracle_b1'][-1]['s_per_iter'] * 1e3:.1f} ms/iter")

    def summary(rows):
        if not rows:
            return None
        out = {"runs": rows}
        for key in ("s_per_iter", "test_rmse", "epochs"):
            if key in rows[0]:
                v = np.array([r[key] for r in rows], dtype=np.float64)
                out[key + "_mean"] = float(v.mean())
                out[key + "_sd"] = float(v.std(ddof=1)) if len(v) > 1 else 0.0
        return out

    out = {"workload": "6040 users x 3883 items, 1,000,209 ratings (80/20 split), k=13, seeds %s" % (seeds,),
           "delta": configs.PAPER_DELTA, "hp": list(configs.PAPER_HP),
           "paper_table1_ml1m_context": {"SVD_s_per_iter": 49.56, "BCSVD_s_per_iter": 34.53,
                                         "BGSVD_s_per_iter": 13.45, "SVD_test_rmse": 0.867,
                                         "BCSVD_test_rmse": 0.871, "BGSVD_test_rmse": 0.869,
                                         "hardware": "Xeon E5-2640 v3 / Tesla M40, MovieLens-1M"}}
    for key, rows in runs.items():
        out[key] = summary(rows)
    out["b3072_graph_identical"] = bool(all(g["epochs"] == d["epochs"] and g["test_rmse"] == d["test_rmse"]
                                            for g, d in zip(runs["gpu_b3072_graph"], runs["gpu_b3072"])))
    if runs["oracle_b8"]:
        out["b8_matched"] = bool(all(abs(g["epochs"] - o["epochs"]) <= 1 and abs(g["test_rmse"] - o["test_rmse"]) <= 1e-3
                                     for g, o in zip(runs["gpu_b8"], runs["oracle_b8"])))
    return out


def incremental_leg(binding, args):
    """Section 6's incremental data on the MovieLens-1M-shaped workload: the
    first 90% of users and items form the old model (fitted to the stopping
    rule), the remaining ratings arrive later (new users, new items and new
    ratings between them and the old ones).  Incremental: bmf_add_ratings
    (5 epochs on the new ratings alone) then the fit on the union, from the
    old factors.  Scratch: the fit on the union from initial values.  Reports
    wall time and test RMSE of both."""
    from paper_1907_07410_amd import configs
    c = configs.PAPER_ML1M
    prob = c.generate(args.seed)
    tr, te = prob.train, prob.test
    m0, n0 = int(prob.m * 0.9), int(prob.n * 0.9)
    old = (tr.u < m0) & (tr.i < n0)
    hp, delta = configs.PAPER_HP, configs.PAPER_DELTA
    G = binding.Model(m0, n0, c.k, 8, seed=args.seed + 1000, order_mode=0)
    G.load_ratings(tr.u[old], tr.i[old], tr.r[old])
    e_old, _ = G.fit(hp, 1000, delta)
    G.synchronize()
    t0 = time.perf_counter()
    G.add_ratings(prob.m, prob.n, tr.u[~old], tr.i[~old], tr.r[~old], hp, 5)
    G.synchronize()
    add_s = time.perf_counter() - t0
    e_inc, _ = G.fit(hp, 1000, delta)
    inc_s = time.perf_counter() - t0
    inc_rmse = G.rmse(te.u, te.i, te.r)
    del G
    S = binding.Model(prob.m, prob.n, c.k, 8, seed=args.seed + 1000, order_mode=0)
    S.load_ratings(np.concatenate([tr.u[old], tr.u[~old]]), np.concatenate([tr.i[old], tr.i[~old]]),
                   np.concatenate([tr.r[old], tr.r[~old]]))
    S.synchronize()
    t0 = time.perf_counter()
    e_s, _ = S.fit(hp, 1000, delta)
    scratch_s = time.perf_counter() - t0
    out = {"old": {"users": m0, "items": n0, "ratings": int(old.sum()), "epochs": e_old},
           "new_ratings": int((~old).sum()),
           "incremental": {"add_ratings_s": add_s, "union_epochs": e_inc, "total_s": inc_s,
                           "test_rmse": inc_rmse},
           "scratch": {"epochs": e_s, "total_s": scratch_s, "test_rmse": S.rmse(te.u, te.i, te.r)}}
    log(f"incremental: add {add_s * 1e3:.1f} ms + {e_inc} union epochs = {inc_s * 1e3:.1f} ms, test rmse "
        f"{inc_rmse:.4f}; scratch {e_s} epochs {scratch_s * 1e3:.1f} ms, test rmse {out['scratch']['test_rmse']:.4f}")
    return out


def out_of_core_leg(binding, args, prob, cfg):
    """The mid workload trained out of core (BMF_OPT_OUT_OF_CORE): ratings
    in pinned host memory, each stratum's plan steps copied to the device
    while the previous ones run.  Reports the load time, the mean of nine
    epochs run back to back and the median of nine epochs each timed on its
    own, against the resident model's, the bytes copied per epoch, and the
    largest
    factor difference against a resident model after two epochs (the same
    kernels; mu differs only by summation order)."""
    tr = prob.train
    G = binding.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0, out_of_core=True)
    t0 = time.perf_counter()
    G.load_ratings(tr.u, tr.i, tr.r)
    load_s = time.perf_counter() - t0
    R = binding.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0)
    R.load_ratings(tr.u, tr.i, tr.r)
    for _ in range(2):
        G.epoch(cfg.lr, cfg.reg)
        R.epoch(cfg.lr, cfg.reg)
    a, b = G.get_factors(), R.get_factors()
    diff = float(max(np.abs(x - y).max() for x, y in zip(a[:4], b[:4])))
    reps = 9

    def epoch_ms(M):
        # nine epochs back to back (one synchronisation at the end: the
        # copies of an epoch's first strata overlap the previous epoch), then
        # nine each timed on its own (synchronised before and after, so the
        # first copy is exposed and a single slow launch shows as one slow
        # epoch): the mean of the first, the median of the second
        M.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            M.epoch(cfg.lr, cfg.reg)
        M.synchronize()
        mean = (time.perf_counter() - t0) / reps * 1e3
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            M.epoch(cfg.lr, cfg.reg)
            M.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
        return mean, float(np.median(t)), t

    res_ms, res_med, res_t = epoch_ms(R)
    del R
    ms, med, t_ooc = epoch_ms(G)
    # bytes copied per epoch: the plan steps (four 16-byte slot records each)
    # and one block table per stratum
    kern, steps, _ = G.plan_info()
    copied = steps * 64 + cfg.b * (cfg.b + 1) * 8
    out = {"load_s": load_s, "ms_per_epoch": ms, "resident_ms_per_epoch": res_ms, "kernel": kern,
           "slowdown_vs_resident": ms / res_ms, "median_ms_per_epoch": med, "resident_median_ms_per_epoch": res_med,
           "median_slowdown_vs_resident": med / res_med, "epochs_timed": reps,
           "synchronised_epoch_ms": t_ooc, "resident_synchronised_epoch_ms": res_t, "h2d_bytes_per_epoch": copied,
           "h2d_GBps_needed": copied / (ms / 1e3) / 1e9, "max_abs_diff_vs_resident_2_epochs": diff}
    log(f"out of core: load {load_s:.2f}s, {ms:.2f} ms/epoch back to back, {med:.2f} median synchronised "
        f"(resident {res_ms:.2f} / {res_med:.2f}), {copied / 1e6:.0f} MB copied per epoch, diff vs resident {diff:.2g}")
    return out


def block_depths(u, i, m, n, b, perm, bp, binding):
    """Dependency depth of every block (bmf_chain_depth on the block's
    ratings in processing order, local ids), as a b x b array."""
    rb, cb = -(-m // b), -(-n // b)
    out = np.zeros(b * b, dtype=np.int64)
    up, ip = u[perm], i[perm]
    for q in range(b * b):
        a, e = int(bp[q]), int(bp[q + 1])
        if e > a:
            br, bc = divmod(q, b)
            out[q] = binding.chain_depth(up[a:e] - br * rb, ip[a:e] - bc * cb)
    return out.reshape(b, b)


def stratum_sum_of_max(x, b):
    """Sum over strata s of the largest entry of blocks ((j + s) mod b, j)."""
    return int(sum(max(int(x[(j + s) % b, j]) for j in range(b)) for s in range(b)))


def train_leg(binding, args, torch, cfg, steps, warmup, cpu_epochs, copy_gbps):
    """One configuration trained and timed: load, a warm-up epoch compared
    with the oracle's first epoch, `steps` timed steps (epoch + test RMSE on
    device-resident test ratings), the HBM and dependency-chain views of the
    SGD stratum kernel, the oracle's epochs on the host cores (the CPU
    baseline), and a second GPU model trained the configuration's epochs whose
    test RMSE is compared with the oracle's after the same epochs."""
    t0 = time.time()
    prob = cfg.generate(args.seed)
    tr, te = prob.train, prob.test
    log(f"{cfg.name}: generated {len(tr)} train / {len(te)} test ratings in {time.time() - t0:.1f}s")
    abytes, nu_blk, ni_blk = algorithmic_bytes(tr.u, tr.i, prob.m, prob.n, cfg.b, cfg.k)
    cp, maxblk, meanblk = critical_path(tr.u, tr.i, prob.m, prob.n, cfg.b)
    log(f"{cfg.name}: algorithmic bytes/epoch {abytes / 1e9:.3f} GB; largest blocks {cp} ratings per epoch")
    G = binding.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0,
                      order_seed=args.seed + 2000, sgd_kernel=args.sgd_kernel)
    t0 = time.time()
    G.load_ratings(tr.u, tr.i, tr.r)
    load_s = time.time() - t0
    log(f"{cfg.name}: load + partition + plan {load_s:.2f}s")
    G.epoch(cfg.lr, cfg.reg)
    G.synchronize()
    parity = cpu = match = None
    threads = max(1, min(len(os.sched_getaffinity(0)), 64))
    if cpu_epochs > 0:
        import oracle
        O = oracle.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0)
        O.load(tr.u, tr.i, tr.r)
        t0 = time.time()
        O.epoch(cfg.lr, cfg.reg, threads=threads)
        first_s = time.time() - t0
        P, Q, bu, bi, mu = G.get_factors()
        parity = float(max(np.abs(P - O.P).max(), np.abs(Q - O.Q).max(), np.abs(bu - O.bu).max(),
                           np.abs(bi - O.bi).max()))
        del P, Q
        log(f"{cfg.name}: oracle epoch {first_s:.1f}s on {threads} threads; 1-epoch max abs diff {parity:.3g}")
        # the configuration's epochs on both sides: matched RMSE
        G2 = binding.Model(prob.m, prob.n, cfg.k, cfg.b, seed=args.seed + 1000, order_mode=0)
        G2.load_ratings(tr.u, tr.i, tr.r)
        for _ in range(cfg.epochs):
            G2.epoch(cfg.lr, cfg.reg)
        t0 = time.time()
        for _ in range(cpu_epochs - 1):
            O.epoch(cfg.lr, cfg.reg, threads=threads)
        cpu_s = first_s + time.time() - t0
        if cpu_epochs == cfg.epochs:
            g_te, o_te = G2.rmse(te.u, te.i, te.r), O.rmse(te.u, te.i, te.r)
            match = {"epochs": cfg.epochs, "gpu_test_rmse": g_te, "oracle_test_rmse": o_te,
                     "abs_diff": abs(g_te - o_te), "matched": bool(abs(g_te - o_te) <= 1e-3)}
            log(f"{cfg.name}: {cfg.epochs} epochs test rmse gpu {g_te:.6f} oracle {o_te:.6f}")
        del O, G2
        cpu = {"value": len(tr) * cpu_epochs / cpu_s, "unit": "rating updates/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{cpu_epochs} full epochs of this workload ({len(tr)} updates each, FP64, "
                         f"{threads} threads over each stratum's blocks), {cpu_s:.1f}s"}
        log(f"{cfg.name}: oracle {cpu_epochs} epochs {cpu_s:.1f}s on {threads} threads")
    for _ in range(warmup - 1):
        G.epoch(cfg.lr, cfg.reg)
    G.synchronize()
    G.sgd_timing(reset=True)
    # test ratings resident on the device for the timed steps
    tu = torch.from_numpy(te.u).cuda()
    ti = torch.from_numpy(te.i).cuda()
    tr_ = torch.from_numpy(te.r).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rmse = None
    for _ in range(steps):
        G.epoch(cfg.lr, cfg.reg)
        rmse = G.rmse_dev(tu, ti, tr_)
    G.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sgd_ms, launches = G.sgd_timing(reset=True)
    per_launch_ms = sgd_ms / max(1, launches)
    achieved = (abytes / cfg.b) / (per_launch_ms / 1e3) / 1e9
    log(f"{cfg.name}: {steps} steps in {el:.3f}s ({len(tr) * steps / el / 1e6:.0f}M updates/s); sgd kernels "
        f"{sgd_ms:.2f} ms over {launches} launches ({per_launch_ms * 1e3:.1f} us each); test rmse {rmse:.4f}")
    # the dependency-chain view of the same launches: every block runs its
    # plan's steps (four independent ratings each) one after another, and a
    # stratum lasts as long as its longest block; the floor is the time of one
    # dependent step of the same step code alone on one wavefront
    kern, plan_steps, slots, blk_steps = G.plan_info(per_block=True)
    crit_steps = stratum_sum_of_max(blk_steps, cfg.b)
    bp, perm = G.get_partition(len(tr))
    depth = block_depths(tr.u, tr.i, prob.m, prob.n, cfg.b, perm, bp, binding)
    dag = stratum_sum_of_max(depth, cfg.b)
    floor_ns = binding.chain_floor_ns(cfg.k)
    epoch_kernel_ms = per_launch_ms * cfg.b
    chain = {"kernel": kern, "plan_steps_per_epoch": plan_steps, "ratings_per_step": len(tr) / max(1, plan_steps),
             "lds_user_slots": slots, "critical_steps_per_epoch": crit_steps,
             "dependency_depth_per_epoch": dag, "floor_ns_per_step": floor_ns,
             "floor_ms_per_epoch": crit_steps * floor_ns / 1e6,
             "depth_floor_ms_per_epoch": dag * floor_ns / 1e6,
             "kernel_ms_per_epoch": epoch_kernel_ms,
             "ns_per_critical_step": epoch_kernel_ms * 1e6 / max(1, crit_steps),
             "frac": crit_steps * floor_ns / 1e6 / epoch_kernel_ms}
    log(f"{cfg.name}: chain {crit_steps} critical plan steps per epoch (dependency depth {dag}), "
        f"{chain['ns_per_critical_step']:.0f} ns each against a {floor_ns:.0f} ns dependent-step floor")
    # test-RMSE pass alone, timed with events on a named stream the library
    # enqueues on: algorithmic bytes = the COO once (12 B) plus the user and
    # item rows with biases ((k+1) 4 B each) per rating
    G.synchronize()
    ts = torch.cuda.Stream()
    G.set_option(binding.OPT_STREAM, ts.cuda_stream)
    G.rmse_dev(tu, ti, tr_)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ev0.record(ts)
    for _ in range(reps):
        G.rmse_dev(tu, ti, tr_)
    ev1.record(ts)
    ts.synchronize()
    rmse_ms = ev0.elapsed_time(ev1) / reps
    rmse_bytes = len(te) * (12 + 2 * (cfg.k + 1) * 4)
    rmse_out = {"ratings": len(te), "ms": rmse_ms, "algorithmic_bytes": rmse_bytes,
                "achieved_GBps": rmse_bytes / (rmse_ms / 1e3) / 1e9,
                "frac_of_hbm_peak": rmse_bytes / (rmse_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                "note": "includes the device range check and the FP64 partial-sum tree"}
    G.set_option(binding.OPT_STREAM, 0)
    log(f"{cfg.name}: test RMSE pass {rmse_ms:.3f} ms, {rmse_out['achieved_GBps']:.0f} GB/s algorithmic")
    out = {"workload": f"{cfg.name}: {prob.m} users x {prob.n} items, {len(tr)} training ratings, k={cfg.k}, "
                       f"{cfg.b}x{cfg.b} blocks, lr {cfg.lr}, reg {cfg.reg}",
           "m": prob.m, "n": prob.n, "n_train": len(tr), "n_test": len(te), "k": cfg.k, "b": cfg.b,
           "updates_per_s": len(tr) * steps / el, "ms_per_step": el / steps * 1e3, "steps": steps,
           "rmse_test": rmse, "parity_1epoch_max_abs": parity, "rmse_match": match, "cpu_baseline": cpu,
           "load_s": load_s, "largest_blocks_ratings_per_epoch": cp, "block_ratings_max": maxblk,
           "block_ratings_mean": meanblk,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg.name),
                        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                        "kernel": "sgd stratum kernel (sgd_plan_kernel)", "algorithmic_bytes_per_launch": abytes / cfg.b,
                        "algorithmic_bytes_per_epoch": abytes, "avg_launch_ms": per_launch_ms,
                        "copy_kernel_GBps": copy_gbps, "chain": chain},
           "rmse_pass": rmse_out}
    return out, G, prob


def tuned_grid_leg(binding, args, torch, cfg, prob, with_oracle):
    """The same workload on the block grid the library's autotuner picks for
    it (a batch of one problem created without a grid: the cost model of the
    dependency chain and block staging, fitted from timed epochs), trained
    for the configuration's epochs through the batch's launches (one per
    stratum).  Epochs 2 to the last are timed; the test RMSE after the last
    is compared with the FP64 oracle's on the same grid, the same schedule
    and the same initial values."""
    tr, te = prob.train, prob.test
    bt = binding.Batch([(prob.m, prob.n)], cfg.k, seed=args.seed + 1000)
    bt.load(0, tr.u, tr.i, tr.r)
    t0 = time.time()
    bt.tune()
    tune_s = time.time() - t0
    b, waves, predicted = bt.info(0)
    bt.epochs(1, cfg.lr, cfg.reg)
    bt.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.epochs(cfg.epochs - 1, cfg.lr, cfg.reg)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, launches = bt.timing(reset=True)
    G = bt.problem(0)
    g_te = G.rmse(te.u, te.i, te.r)
    abytes, _, _ = algorithmic_bytes(tr.u, tr.i, prob.m, prob.n, b, cfg.k)
    out = {"b": b, "waves": waves, "tune_s": tune_s, "model_ms_per_epoch": predicted,
           "updates_per_s": len(tr) * (cfg.epochs - 1) / el, "ms_per_epoch": el / (cfg.epochs - 1) * 1e3,
           "kernel_ms_per_epoch": ms / (cfg.epochs - 1), "launches_per_epoch": launches / (cfg.epochs - 1),
           "algorithmic_bytes_per_epoch": abytes,
           "achieved_GBps": abytes / (ms / (cfg.epochs - 1) / 1e3) / 1e9,
           "gpu_test_rmse": g_te}
    out["frac_of_hbm_peak"] = out["achieved_GBps"] / HBM_PEAK_GBS
    if with_oracle:
        import oracle
        threads = max(1, min(len(os.sched_getaffinity(0)), 64))
        O = oracle.Model(prob.m, prob.n, cfg.k, b, seed=args.seed + 1000, order_mode=0)
        O.load(tr.u, tr.i, tr.r)
        for _ in range(cfg.epochs):
            O.epoch(cfg.lr, cfg.reg, threads=threads)
        o_te = O.rmse(te.u, te.i, te.r)
        out["rmse_match"] = {"epochs": cfg.epochs, "gpu_test_rmse": g_te, "oracle_test_rmse": o_te,
                             "abs_diff": abs(g_te - o_te), "matched": bool(abs(g_te - o_te) <= 1e-3)}
        del O
    log(f"{cfg.name}: autotuned grid {b}x{b} ({waves} waves, tuned in {tune_s:.1f}s): "
        f"{out['updates_per_s'] / 1e6:.0f}M updates/s, {out['ms_per_epoch']:.2f} ms/epoch, test rmse {g_te:.6f}"
        + (f" (oracle {out['rmse_match']['oracle_test_rmse']:.6f})" if with_oracle else ""))
    bt.close()
    return out


def topk_all_users(binding, torch, G, prob, cfg):
    """Top-100 for every user in FP32 and in BF16 with FP32 rescoring (GPU
    time with events on the library's stream; contraction FLOPs 2 m n k
    against the MI355X dense matrix peak of each precision), and BF16 recall
    against FP32 on 20,000 of the users."""
    users = torch.arange(prob.m, dtype=torch.int32, device="cuda")
    ts = torch.cuda.Stream()
    G.set_option(binding.OPT_STREAM, ts.cuda_stream)
    flops = 2.0 * prob.m * prob.n * cfg.k
    res = {}
    out = {"users": prob.m, "items": prob.n, "k": cfg.k, "K": 100, "contraction_flop": flops}
    for name, prec, peak in (("fp32", 0, MFMA_PEAK_TFLOPS["fp32"]), ("bf16", 1, MFMA_PEAK_TFLOPS["bf16"])):
        it = torch.empty((prob.m, 100), dtype=torch.int32, device="cuda")
        sc = torch.empty((prob.m, 100), dtype=torch.float32, device="cuda")
        G.topk_dev(users, 100, prec, 0, it, sc)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(ts)
        G.topk_dev(users, 100, prec, 0, it, sc)
        ev1.record(ts)
        ts.synchronize()
        dt = ev0.elapsed_time(ev1) / 1e3
        res[name] = it[:20000].cpu().numpy()
        out[f"{name}_ms"] = dt * 1e3
        out[f"{name}_users_per_s"] = prob.m / dt
        out[f"{name}_tflops"] = flops / dt / 1e12
        out[f"{name}_frac_of_mfma_peak"] = flops / dt / 1e12 / peak
        del it, sc
    G.set_option(binding.OPT_STREAM, 0)
    out["recall_at_100_bf16_vs_fp32_20k_users"] = float(
        np.mean([len(set(a) & set(b)) / 100 for a, b in zip(res["fp32"], res["bf16"])]))
    log(f"{cfg.name}: top-100 for all {prob.m} users FP32 {out['fp32_ms']:.1f} ms "
        f"({out['fp32_frac_of_mfma_peak'] * 100:.1f}% of peak), BF16 {out['bf16_ms']:.1f} ms "
        f"({out['bf16_frac_of_mfma_peak'] * 100:.1f}%), recall {out['recall_at_100_bf16_vs_fp32_20k_users']:.6f}")
    return out


def topk_batch(binding, torch, G, prob, cfg, nusers, seed):
    """Top-100 for a batch of users in FP32 and BF16 scoring (GPU time with
    events), recall of BF16 against FP32 and of both against FP64 scores of
    the same factors on 64 of the users, and one small request's latency."""
    rng = np.random.default_rng(seed)
    users = rng.integers(0, prob.m, nusers).astype(np.int32)
    topk = {}
    res = {}
    du = torch.from_numpy(users).cuda()
    torch.cuda.synchronize()
    ts = torch.cuda.Stream()
    G.set_option(binding.OPT_STREAM, ts.cuda_stream)
    flops = 2.0 * len(users) * prob.n * cfg.k
    for name, prec, peak in (("fp32", 0, MFMA_PEAK_TFLOPS["fp32"]), ("bf16", 1, MFMA_PEAK_TFLOPS["bf16"])):
        it = torch.empty((len(users), 100), dtype=torch.int32, device="cuda")
        sc = torch.empty((len(users), 100), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        G.topk_dev(du, 100, prec, 0, it, sc)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        ev0.record(ts)
        for _ in range(reps):
            G.topk_dev(du, 100, prec, 0, it, sc)
        ev1.record(ts)
        ts.synchronize()
        dt = ev0.elapsed_time(ev1) / reps / 1e3
        res[name] = (it.cpu().numpy(), sc.cpu().numpy())
        topk[name + "_users_per_s"] = len(users) / dt
        topk[name + "_ms"] = dt * 1e3
        topk[name + "_contraction_tflops"] = flops / dt / 1e12
        topk[name + "_frac_of_mfma_peak"] = flops / dt / 1e12 / peak
    G.set_option(binding.OPT_STREAM, 0)
    topk["recall_at_100_bf16_vs_fp32"] = float(
        np.mean([len(set(a) & set(b)) / 100 for a, b in zip(res["fp32"][0], res["bf16"][0])]))
    P, Q, bu, bi, mu = G.get_factors()
    Qd, bid = Q.astype(np.float64), bi.astype(np.float64)
    rec = {"fp32": [], "bf16": []}
    err = {"fp32": 0.0, "bf16": 0.0}
    for row in range(64):
        uu = users[row]
        s64 = mu + float(bu[uu]) + bid + Qd @ P[uu].astype(np.float64)
        best = set(np.argsort(-s64, kind="stable")[:100].tolist())
        for name in ("fp32", "bf16"):
            its, scs = res[name][0][row], res[name][1][row]
            rec[name].append(len(best & set(its.tolist())) / 100)
            err[name] = max(err[name], float(np.abs(scs.astype(np.float64) - s64[its]).max()))
    for name in ("fp32", "bf16"):
        topk[f"recall_at_100_{name}_vs_fp64"] = float(np.mean(rec[name]))
        topk[f"max_score_error_{name}_vs_fp64"] = err[name]
    topk["users"] = len(users)
    topk["items"] = prob.n
    small = {}
    G.set_option(binding.OPT_STREAM, ts.cuda_stream)
    for nb in (1, 16, 64):
        du_s = du[:nb].contiguous()
        it = torch.empty((nb, 100), dtype=torch.int32, device="cuda")
        sc = torch.empty((nb, 100), dtype=torch.float32, device="cuda")
        row = {}
        for name, prec in (("fp32", 0), ("bf16", 1)):
            G.topk_dev(du_s, 100, prec, 0, it, sc)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(ts)
            for _ in range(10):
                G.topk_dev(du_s, 100, prec, 0, it, sc)
            ev1.record(ts)
            ts.synchronize()
            row[name + "_ms"] = ev0.elapsed_time(ev1) / 10
        small[str(nb)] = row
    G.set_option(binding.OPT_STREAM, 0)
    topk["small_batches"] = small
    log(f"{cfg.name}: top-100 for {len(users)} users FP32 {topk['fp32_ms']:.3f} ms, BF16 {topk['bf16_ms']:.3f} ms, "
        f"recall {topk['recall_at_100_bf16_vs_fp32']:.4f}")
    return topk


def copy_bandwidth(torch):
    """A plain device copy (1 GiB read + 1 GiB written): the streaming rate
    the chip delivers next to the datasheet peak."""
    xb = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    yb = torch.empty_like(xb)
    yb.copy_(xb)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        yb.copy_(xb)
    ev1.record()
    torch.cuda.synchronize()
    gbps = 2 * xb.numel() * 4 * 5 / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del xb, yb
    log(f"device copy (1 GiB read + 1 GiB written): {gbps:.0f} GB/s")
    return gbps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--topk-users", type=int, default=4096, help="users of the mid workload's top-K batch (0 skips)")
    ap.add_argument("--sgd-kernel", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests per serving measurement (0 skips the serving leg)")
    ap.add_argument("--batched-scale", type=float, default=1.0,
                    help="linear scale of the 64-problem batched workload's m and n (0 skips the batched leg)")
    ap.add_argument("--no-paper-protocol", action="store_true",
                    help="skip the MovieLens-1M-shaped early-termination and incremental legs")
    ap.add_argument("--no-out-of-core", action="store_true", help="skip the out-of-core leg")
    ap.add_argument("--no-mid", action="store_true", help="skip the mid workload's leg (and the out-of-core leg)")
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline workload's leg alone (for profiling runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (there is no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.warmup < 1:
        args.warmup = 1
    if args.headline_only:
        args.no_mid = args.no_out_of_core = args.no_paper_protocol = True
        args.serving_requests = 0
        args.batched_scale = 0.0

    import torch
    from paper_1907_07410_amd import binding, configs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    copy_gbps = copy_bandwidth(torch)
    cfg = configs.LARGE
    cpu_epochs = 0 if args.no_cpu_baseline else cfg.epochs
    head, G, prob = train_leg(binding, args, torch, cfg, args.steps, args.warmup, cpu_epochs, copy_gbps)
    head["topk_all_users"] = topk_all_users(binding, torch, G, prob, cfg)
    G.close()
    del G
    if not args.headline_only:
        head["tuned_grid"] = tuned_grid_leg(binding, args, torch, cfg, prob, not args.no_cpu_baseline)
    del prob
    mid = None
    ooc_out = None
    if not args.no_mid:
        mcfg = configs.MID
        mid, Gm, mprob = train_leg(binding, args, torch, mcfg, args.steps, 1,
                                   0 if args.no_cpu_baseline else mcfg.epochs, copy_gbps)
        if args.topk_users > 0:
            mid["topk"] = topk_batch(binding, torch, Gm, mprob, mcfg, args.topk_users, 7)
        Gm.close()
        del Gm
        mid["tuned_grid"] = tuned_grid_leg(binding, args, torch, mcfg, mprob, not args.no_cpu_baseline)
        ooc_out = None if args.no_out_of_core else out_of_core_leg(binding, args, mprob, mcfg)
        del mprob
    serving_out = serving_leg(binding, args) if args.serving_requests > 0 else None
    batched_out = batched_leg(binding, args, torch) if args.batched_scale > 0 else None
    paper_out = None if args.no_paper_protocol else paper_leg(binding, args)
    incr_out = None if args.no_paper_protocol else incremental_leg(binding, args)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x (read {nbytes} B, write {nbytes} B) elementwise kernel")
        del x, y

    line = {
        "metric": "rating updates/s at matched RMSE; top-100 req/s + p99 latency (BF16 vs FP32)",
        "value": head["updates_per_s"],
        "unit": "rating updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large-scale: 480000 users x 17800 items, 100M Zipf(1.0) integer ratings "
                               "(90M train), k=128, 128x128 blocks, lr 0.005, reg 0.05",
                   "m": head["m"], "n": head["n"], "n_train": head["n_train"], "k": head["k"], "b": head["b"]},
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "rmse_test": head["rmse_test"],
        "parity_1epoch_max_abs": head["parity_1epoch_max_abs"],
        "rmse_match": head["rmse_match"],
        "load_s": head["load_s"],
        "rmse_pass": head["rmse_pass"],
        "topk_all_users": head["topk_all_users"],
        "tuned_grid": head.get("tuned_grid"),
        "mid": mid,
        "serving": serving_out,
        "batched": batched_out,
        "paper_protocol": paper_out,
        "incremental": incr_out,
        "out_of_core": ooc_out,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
