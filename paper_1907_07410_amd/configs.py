"""The five synthetic workloads, made concrete.

tiny     1,000 x 500, 20,000 uniform cells, planted rank 8, k=16, b=4
mid      138,000 x 27,000, 20M ratings, Zipf(1.1), half stars, k=64, b=64
large    480,000 x 17,800, 100M ratings, Zipf(1.0), integers, k=128, b=128
batched  64 problems, 10k-200k x 2k-50k, density 0.1-1%, k=32, 10 epochs
serving  1M x 100k factor tables, k=128, BF16 scoring copy
paper    6,040 x 3,883 (the MovieLens-1M shape of Section 5), 1,000,209 ratings,
         80/20 split, k=13, the four named (alpha, beta) pairs, delta = 1e-4

Seeds: data seed s (default 1), model seed s+1000, schedule seed s+2000.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import synth


@dataclass
class TrainConfig:
    name: str
    m: int
    n: int
    nnz: int            # total ratings before the split
    k: int
    b: int
    lr: float
    reg: float
    epochs: int
    rank: int
    noise: float
    rounding: str
    zipf_user: Optional[float]   # None -> uniform random cells
    zipf_item: Optional[float]
    train_frac: float = 1.0
    sigma_f: float = 0.3
    offset: float = 3.5
    seeded_order: bool = True    # seeded stratum order per epoch

    def generate(self, seed: int = 1, scale: float = 1.0) -> synth.Problem:
        """Draw the workload.  ``scale`` < 1 shrinks m, n and nnz by the same
        factor (density preserved) for quick tests."""
        m = max(1, int(round(self.m * scale)))
        n = max(1, int(round(self.n * scale)))
        nnz = max(1, int(round(self.nnz * scale)))
        nnz = min(nnz, m * n)
        rng = np.random.default_rng(seed)
        if self.zipf_user is None:
            u, i = synth.sample_pairs_uniform(m, n, nnz, rng)
        else:
            u, i = synth.sample_pairs_zipf(m, n, nnz, self.zipf_user, self.zipf_item, rng)
        r = synth.planted_values(u, i, m, n, self.rank, self.sigma_f, self.noise,
                                 self.offset, self.rounding, rng)
        rat = synth.Ratings(u, i, r)
        if self.train_frac < 1.0:
            tr, te = synth.split(rat, self.train_frac, rng)
            return synth.Problem(m, n, tr, te)
        return synth.Problem(m, n, rat, None)


TINY = TrainConfig("tiny", 1000, 500, 20000, k=16, b=4, lr=0.01, reg=0.02, epochs=20,
                   rank=8, noise=0.5, rounding="int", zipf_user=None, zipf_item=None)
MID = TrainConfig("mid", 138000, 27000, 20_000_000, k=64, b=64, lr=0.005, reg=0.05,
                  epochs=20, rank=32, noise=0.7, rounding="half", zipf_user=1.1,
                  zipf_item=1.1, train_frac=0.9, seeded_order=False)
LARGE = TrainConfig("large", 480000, 17800, 100_000_000, k=128, b=128, lr=0.005, reg=0.05,
                    epochs=20, rank=64, noise=0.9, rounding="int", zipf_user=1.0,
                    zipf_item=1.0, train_frac=0.9, seeded_order=False)


# Section 5's protocol on synthetic ratings of the MovieLens-1M shape: 6,040
# users, 3,883 items (ceil(n / 8) = 486, the block width the paper states for
# its 8 x 8 grid), 1,000,209 ratings, integer stars, an 80/20 split, k = 13
# and the (alpha, beta) pairs the paper gives by name, early termination when
# the training RMSE improves by less than 1e-4.  Zipf exponents 0.35 (users:
# degrees 108 to 2,271) and 0.5 (items: 131 to 6,040) keep the capped degrees
# close to the spread of that data set; planted factors N(0, 0.45^2) of rank 13
# and noise 0.8 give ratings of standard deviation about 1.04 and a test RMSE
# near 0.88 at the stopping epoch, the regime of the paper's Table 1.  Grids: 1
# (the plain method), 8 (the paper's CPU block variant) and 3072 (its GPU
# variant).
PAPER_ML1M = TrainConfig("paper", 6040, 3883, 1_000_209, k=13, b=8, lr=0.0, reg=0.0, epochs=300,
                         rank=13, noise=0.8, rounding="int", zipf_user=0.35, zipf_item=0.5,
                         train_frac=0.8, sigma_f=0.45, seeded_order=False)
# {alpha_p, beta_p, alpha_q, beta_q, alpha_bu, beta_bu, alpha_bi, beta_bi}
PAPER_HP = (0.019, 0.019, 0.004, 0.019, 0.004, 0.019, 0.013, 0.007)
PAPER_DELTA = 1e-4
PAPER_GRIDS = (1, 8, 3072)


@dataclass
class BatchedConfig:
    nprob: int = 64
    m_range: tuple = (10_000, 200_000)
    n_range: tuple = (2_000, 50_000)
    density: tuple = (0.001, 0.01)
    k: int = 32
    lr: float = 0.01
    reg: float = 0.02
    epochs: int = 10
    rank: int = 16
    noise: float = 0.5

    def shapes(self, seed: int = 1, scale: float = 1.0):
        rng = np.random.default_rng(seed)
        out = []
        for _ in range(self.nprob):
            m = int(rng.integers(self.m_range[0], self.m_range[1] + 1))
            n = int(rng.integers(self.n_range[0], self.n_range[1] + 1))
            d = float(rng.uniform(*self.density))
            m2 = max(8, int(round(m * scale)))
            n2 = max(8, int(round(n * scale)))
            out.append((m2, n2, max(1, int(round(d * m2 * n2)))))
        return out

    def generate(self, seed: int = 1, scale: float = 1.0, workers: int = 1,
                 progress=None) -> List[synth.Problem]:
        """The problems at ``scale``.  Problem p draws from its own generator
        (seed * 1000 + p), so ``workers`` threads give the same data as one;
        numpy's sorting and sampling release the interpreter lock, which is
        what lets threads help (the full size is about 1e9 ratings).
        ``progress(p)``, if given, is called as problem p is finished."""
        shapes = self.shapes(seed, scale)

        def one(p: int) -> synth.Problem:
            m, n, nnz = shapes[p]
            rng = np.random.default_rng(seed * 1000 + p)
            # one thread per problem: the problems themselves run in parallel
            u, i = synth.sample_pairs_zipf(m, n, nnz, 1.1, 1.1, rng, workers=1)
            r = synth.planted_values(u, i, m, n, self.rank, 0.3, self.noise, 3.5, "int", rng, workers=1)
            if progress is not None:
                progress(p)
            return synth.Problem(m, n, synth.Ratings(u, i, r), None)

        if workers <= 1:
            return [one(p) for p in range(len(shapes))]
        from concurrent.futures import ThreadPoolExecutor
        # largest problems first, so the longest draw starts at once
        order = sorted(range(len(shapes)), key=lambda p: -shapes[p][2])
        with ThreadPoolExecutor(max_workers=workers) as ex:
            done = dict(zip(order, ex.map(one, order)))
        return [done[p] for p in range(len(shapes))]


BATCHED = BatchedConfig()


@dataclass
class ServingConfig:
    m: int = 1_000_000
    n: int = 100_000
    k: int = 128
    K: int = 100
    topk_frac: float = 0.9
    batch_range: tuple = (1, 4096)
    foldin_range: tuple = (5, 500)
    foldin_passes: int = 10
    lr: float = 0.005
    reg: float = 0.05


SERVING = ServingConfig()

CONFIGS = {"tiny": TINY, "mid": MID, "large": LARGE, "paper": PAPER_ML1M}
