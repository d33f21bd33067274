"""FP64 CPU oracle for block-based biased-SVD SGD (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps ``oracle.c`` (plain C, built with gcc into
``liboracle.so``) through ctypes; it imports nothing from the HIP library.

What pins each part (tests/test_oracle*.py, CPU): SplitMix64 and the BF16
rounding (one value and whole arrays) against published values; the single-rating update and the bias
dynamics against hand and closed-form values; the partition against an
independent lexsort; the schedule against the Latin-square property and the
paper's diagonal-first order; an epoch against the pinned update applied
rating by rating (three update forms: Eqs 10-13, Algorithm 2's factor order,
Algorithm 2 as printed); RMSE against a closed form; the loss against a
closed form and a hand-worked example with every penalty term; top-K, and
the ranking of an explicit user vector, against brute force (and the two
against each other); fold-in against the ridge solution it converges to;
the stopping rule
of Algorithm 1 (``Model.fit``) against a recorded trajectory; incremental
data (``Model.add_ratings``) against growth, untouched-row and partition
invariants.  No function is left without a pin; the paper's own Table 1
figures are the one thing not reproduced (their data sets are not here).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, so every FP64
    operation rounds once as written)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lpthread", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB_PATH)
            i64, i32, u64, dbl, p = C.c_int64, C.c_int32, C.c_uint64, C.c_double, C.c_void_p
            L.orc_splitmix64.restype = u64
            L.orc_splitmix64.argtypes = [u64, u64]
            L.orc_init_value.restype = dbl
            L.orc_init_value.argtypes = [u64, C.c_int, i64, C.c_int, C.c_int]
            L.orc_init_factors.argtypes = [i64, i64, C.c_int, u64, p, p, p, p]
            L.orc_mean.restype = dbl
            L.orc_mean.argtypes = [p, i64]
            L.orc_partition.restype = C.c_int
            L.orc_partition.argtypes = [i64, i64, C.c_int, p, p, i64, p, p]
            L.orc_schedule.argtypes = [C.c_int, u64, C.c_int, C.c_int, p]
            L.orc_epoch.restype = C.c_int
            L.orc_epoch.argtypes = [i64, i64, C.c_int, C.c_int, p, p, p, p, dbl, p, C.c_int,
                                    p, p, p, p, p, p, C.c_int]
            L.orc_rmse.restype = dbl
            L.orc_rmse.argtypes = [C.c_int, p, p, p, p, dbl, p, p, p, i64]
            L.orc_loss.restype = dbl
            L.orc_loss.argtypes = [C.c_int, p, p, p, p, dbl, p, p, p, p, i64]
            L.orc_topk.restype = C.c_int
            L.orc_topk.argtypes = [i64, C.c_int, p, p, p, p, dbl, p, i64, C.c_int, p, p]
            L.orc_topk_vec.restype = C.c_int
            L.orc_topk_vec.argtypes = [i64, C.c_int, p, dbl, p, p, dbl, C.c_int, p, p]
            L.orc_foldin.argtypes = [C.c_int, p, p, dbl, p, p, i64, C.c_int, p, p, p]
            L.orc_bf16_round.restype = C.c_float
            L.orc_bf16_round.argtypes = [C.c_float]
            L.orc_bf16_round_n.argtypes = [p, p, i64]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def hparams(lr: float, reg: float) -> np.ndarray:
    """The eight (alpha, beta) values of Eqs 10-13 set to one (lr, reg)."""
    return np.array([lr, reg] * 4, dtype=np.float64)


def splitmix64(seed: int, j: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed & (2**64 - 1)), C.c_uint64(j)))


def init_value(seed: int, tag: int, row: int, k: int, f: int) -> float:
    return float(lib().orc_init_value(C.c_uint64(seed), tag, row, k, f))


def mean(r) -> float:
    r = _c(r, np.float32)
    return float(lib().orc_mean(_ptr(r), r.shape[0]))


def partition(m: int, n: int, b: int, u, i):
    u = _c(u, np.int32)
    i = _c(i, np.int32)
    bp = np.zeros(b * b + 1, dtype=np.int64)
    perm = np.zeros(u.shape[0], dtype=np.int32)
    rc = lib().orc_partition(m, n, b, _ptr(u), _ptr(i), u.shape[0], _ptr(bp), _ptr(perm))
    if rc != 0:
        raise ValueError("orc_partition failed: %d" % rc)
    return bp, perm


def schedule(b: int, seed: int, epoch: int, mode: int) -> np.ndarray:
    out = np.zeros(b, dtype=np.int32)
    lib().orc_schedule(b, C.c_uint64(seed), epoch, mode, _ptr(out))
    return out


def bf16_round(x: float) -> float:
    return float(lib().orc_bf16_round(C.c_float(x)))


def bf16_round_array(x) -> np.ndarray:
    """bf16_round of every element of an FP32 array (same shape, FP32)."""
    x = _c(x, np.float32)
    y = np.empty_like(x)
    lib().orc_bf16_round_n(_ptr(x), _ptr(y), x.size)
    return y


class Model:
    """FP64 model state plus the operations of the method."""

    def __init__(self, m: int, n: int, k: int, b: int, seed: int = 1001, mu_mode: int = 0,
                 order_mode: int = 0, order_seed: Optional[int] = None):
        self.m, self.n, self.k, self.b = m, n, k, b
        self.seed = seed
        self.order_mode = order_mode
        self.order_seed = seed if order_seed is None else order_seed
        self.mu_mode = mu_mode
        self.P = np.zeros((m, k), dtype=np.float64)
        self.Q = np.zeros((n, k), dtype=np.float64)
        self.bu = np.zeros(m, dtype=np.float64)
        self.bi = np.zeros(n, dtype=np.float64)
        self.mu = 0.0
        self.epoch_no = 0
        lib().orc_init_factors(m, n, k, C.c_uint64(seed), _ptr(self.P), _ptr(self.Q), _ptr(self.bu),
                               _ptr(self.bi))
        self.u = self.i = self.r = None

    def load(self, u, i, r):
        self.u = _c(u, np.int32)
        self.i = _c(i, np.int32)
        self.r = _c(r, np.float32)
        self.mu = mean(self.r) if self.mu_mode == 0 else 0.0
        self.block_ptr, self.perm = partition(self.m, self.n, self.b, self.u, self.i)

    def set_factors(self, P, Q, bu, bi, mu=None):
        self.P[...] = P
        self.Q[...] = Q
        self.bu[...] = bu
        self.bi[...] = bi
        if mu is not None:
            self.mu = float(mu)

    def order(self, epoch: int) -> np.ndarray:
        return schedule(self.b, self.order_seed, epoch, self.order_mode)

    def epoch(self, lr: float = None, reg: float = None, hp: Sequence[float] = None,
              threads: int = 1, gauss_seidel: bool = False, alg2_literal: bool = False):
        """One epoch.  Update form: simultaneous Eqs 10-13 (default);
        ``gauss_seidel``: item factors from the updated user factors;
        ``alg2_literal``: Algorithm 2 as printed (crossed bias regularisers,
        the item bias penalised by the updated user bias, Gauss-Seidel
        factors)."""
        hp = hparams(lr, reg) if hp is None else _c(hp, np.float64)
        order = self.order(self.epoch_no)
        form = 2 if alg2_literal else (1 if gauss_seidel else 0)
        rc = lib().orc_epoch(self.m, self.n, self.k, self.b, _ptr(self.P), _ptr(self.Q), _ptr(self.bu),
                             _ptr(self.bi), self.mu, _ptr(hp), form, _ptr(self.u),
                             _ptr(self.i), _ptr(self.r), _ptr(self.block_ptr), _ptr(self.perm),
                             _ptr(order), threads)
        if rc != 0:
            raise RuntimeError("orc_epoch failed: %d" % rc)
        self.epoch_no += 1

    def fit(self, hp: Sequence[float], max_epochs: int, delta: float, threads: int = 1):
        """Algorithm 1's loop: epochs until the training RMSE improves by
        less than delta over the previous epoch (the first epoch compares with
        the RMSE of the initial factors), at most max_epochs.  Returns
        (epochs run, final training RMSE)."""
        prev = self.rmse()
        done = 0
        while done < max_epochs:
            self.epoch(hp=hp, threads=threads)
            done += 1
            cur = self.rmse()
            if not (prev - cur >= delta):  # also stops once the RMSE is not a number
                return done, cur
            prev = cur
        return done, prev

    def add_ratings(self, m_new: int, n_new: int, u, i, r, hp: Sequence[float], epochs_new: int,
                    threads: int = 1):
        """Section 6's incremental data: the new ratings form new blocks that
        are factorised on their own, then all ratings train together.  The
        model grows to m_new x n_new (learned rows kept; new rows take the
        initial values of a model created at the new size, biases 0), runs
        epochs_new epochs over the new ratings alone on the grown grid from
        the current factors, and makes the union (loaded ratings, then the
        new ones) the training set.  mu is the union's mean (or 0), used in
        both phases."""
        if m_new < self.m or n_new < self.n:
            raise ValueError("the model can only grow")
        u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
        P = np.zeros((m_new, self.k), dtype=np.float64)
        Q = np.zeros((n_new, self.k), dtype=np.float64)
        bu = np.zeros(m_new, dtype=np.float64)
        bi = np.zeros(n_new, dtype=np.float64)
        lib().orc_init_factors(m_new, n_new, self.k, C.c_uint64(self.seed), _ptr(P), _ptr(Q), _ptr(bu), _ptr(bi))
        P[: self.m] = self.P
        Q[: self.n] = self.Q
        bu[: self.m] = self.bu
        bi[: self.n] = self.bi
        self.m, self.n = m_new, n_new
        self.P, self.Q, self.bu, self.bi = P, Q, bu, bi
        if self.u is None:
            au, ai, ar = u, i, r
        else:
            au = np.concatenate([self.u, u])
            ai = np.concatenate([self.i, i])
            ar = np.concatenate([self.r, r])
        mu = mean(ar) if (self.mu_mode == 0 and ar.shape[0] > 0) else 0.0
        if epochs_new > 0 and u.shape[0] > 0:
            self.load(u, i, r)
            self.mu = mu
            for _ in range(epochs_new):
                self.epoch(hp=hp, threads=threads)
        self.load(au, ai, ar)
        self.mu = mu

    def rmse(self, u=None, i=None, r=None) -> float:
        if u is None:
            u, i, r = self.u, self.i, self.r
        u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
        return float(lib().orc_rmse(self.k, _ptr(self.P), _ptr(self.Q), _ptr(self.bu), _ptr(self.bi),
                                    self.mu, _ptr(u), _ptr(i), _ptr(r), u.shape[0]))

    def loss(self, lr: float = 0.0, reg: float = 0.0, hp=None) -> float:
        hp = hparams(lr, reg) if hp is None else _c(hp, np.float64)
        return float(lib().orc_loss(self.k, _ptr(self.P), _ptr(self.Q), _ptr(self.bu), _ptr(self.bi),
                                    self.mu, _ptr(hp), _ptr(self.u), _ptr(self.i), _ptr(self.r),
                                    self.u.shape[0]))

    def topk(self, users, K: int):
        users = _c(users, np.int32)
        items = np.zeros((users.shape[0], K), dtype=np.int32)
        scores = np.zeros((users.shape[0], K), dtype=np.float64)
        rc = lib().orc_topk(self.n, self.k, _ptr(self.P), _ptr(self.Q), _ptr(self.bu), _ptr(self.bi),
                            self.mu, _ptr(users), users.shape[0], K, _ptr(items), _ptr(scores))
        if rc != 0:
            raise RuntimeError("orc_topk failed")
        return items, scores


def topk_dense(P, Q, bu, bi, mu, users, K):
    """Top-K for explicit FP64 tables (not owned by a Model)."""
    P = _c(P, np.float64)
    Q = _c(Q, np.float64)
    bu = _c(bu, np.float64)
    bi = _c(bi, np.float64)
    users = _c(users, np.int32)
    n, k = Q.shape
    items = np.zeros((users.shape[0], K), dtype=np.int32)
    scores = np.zeros((users.shape[0], K), dtype=np.float64)
    rc = lib().orc_topk(n, k, _ptr(P), _ptr(Q), _ptr(bu), _ptr(bi), float(mu), _ptr(users),
                        users.shape[0], K, _ptr(items), _ptr(scores))
    if rc != 0:
        raise RuntimeError("orc_topk failed")
    return items, scores


def topk_vec(p, bu_u, Q, bi, mu, K):
    p = _c(p, np.float64)
    Q = _c(Q, np.float64)
    bi = _c(bi, np.float64)
    n, k = Q.shape
    items = np.zeros(K, dtype=np.int32)
    scores = np.zeros(K, dtype=np.float64)
    lib().orc_topk_vec(n, k, _ptr(p), float(bu_u), _ptr(Q), _ptr(bi), float(mu), K, _ptr(items),
                       _ptr(scores))
    return items, scores


def rmse_dense(P, Q, bu, bi, mu, u, i, r) -> float:
    P, Q = _c(P, np.float64), _c(Q, np.float64)
    bu, bi = _c(bu, np.float64), _c(bi, np.float64)
    u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
    return float(lib().orc_rmse(P.shape[1], _ptr(P), _ptr(Q), _ptr(bu), _ptr(bi), float(mu), _ptr(u),
                                _ptr(i), _ptr(r), u.shape[0]))


def foldin(Q, bi, mu, items, r, passes: int, lr: float = None, reg: float = None, hp=None):
    Q = _c(Q, np.float64)
    bi = _c(bi, np.float64)
    items = _c(items, np.int32)
    r = _c(r, np.float32)
    hp = hparams(lr, reg) if hp is None else _c(hp, np.float64)
    k = Q.shape[1]
    p = np.zeros(k, dtype=np.float64)
    bu = np.zeros(1, dtype=np.float64)
    lib().orc_foldin(k, _ptr(Q), _ptr(bi), float(mu), _ptr(items), _ptr(r), items.shape[0], passes,
                     _ptr(hp), _ptr(p), _ptr(bu))
    return p, float(bu[0])
