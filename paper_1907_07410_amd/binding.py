"""ctypes binding of libbmf (include/bmf.h).

Argument marshalling only: every step runs in the library's HIP kernels.
The library must have been built (``python -m paper_1907_07410_amd.build``);
importing this module without it raises.  Host arrays are numpy arrays;
device arrays are torch tensors on the context's device (``*_dev`` calls).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmf.so")

BMF_OK, BMF_E_INVAL, BMF_E_RANGE, BMF_E_STATE, BMF_E_NOMEM, BMF_E_DEVICE = 0, -1, -2, -3, -4, -5
(OPT_SEED, OPT_ORDER_SEED, OPT_STRATUM_ORDER, OPT_MU_MODE, OPT_STREAM, OPT_SGD_KERNEL, OPT_WAVES_PER_BLOCK,
 OPT_OUT_OF_CORE, OPT_EPOCH, OPT_EPOCH_GRAPH) = range(10)

_STATUS = {0: "BMF_OK", -1: "BMF_E_INVAL", -2: "BMF_E_RANGE", -3: "BMF_E_STATE", -4: "BMF_E_NOMEM",
           -5: "BMF_E_DEVICE"}


class BmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libbmf.so not built at {LIB_PATH}; run python -m paper_1907_07410_amd.build")
    # PyTorch ships its own HIP runtime with the same soname as the system
    # one; loading torch first makes libbmf bind to that same instance, so
    # one HIP runtime serves both and torch device pointers and streams are
    # valid in the library.  (Loaded the other way round, torch would start
    # a second runtime and see no GPU.)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    i64, i32, f32, dbl, p = C.c_int64, C.c_int32, C.c_float, C.c_double, C.c_void_p
    pp = C.POINTER(C.c_void_p)
    sig = {
        "bmf_create": ([i64, i64, i32, i32, pp], i32),
        "bmf_set_option": ([p, i32, i64], i32),
        "bmf_destroy": ([p], None),
        "bmf_last_error": ([p], C.c_char_p),
        "bmf_synchronize": ([p], i32),
        "bmf_load_ratings": ([p, p, p, p, i64], i32),
        "bmf_load_ratings_dev": ([p, p, p, p, i64], i32),
        "bmf_epoch": ([p, f32, f32], i32),
        "bmf_epoch_hp": ([p, p], i32),
        "bmf_epoch_count": ([p, p], i32),
        "bmf_fit": ([p, p, i32, dbl, p, p], i32),
        "bmf_add_ratings": ([p, i64, i64, p, p, p, i64, p, i32], i32),
        "bmf_plan_info": ([p, p, p, p, p], i32),
        "bmf_get_schedule": ([p, i32, p], i32),
        "bmf_get_partition": ([p, p, p], i32),
        "bmf_get_factors": ([p, p, p, p, p, p], i32),
        "bmf_set_factors": ([p, p, p, p, p, p], i32),
        "bmf_factor_ptrs": ([p, pp, pp, pp, pp], i32),
        "bmf_rmse": ([p, p, p, p, i64, p], i32),
        "bmf_loss": ([p, p, p], i32),
        "bmf_check_disjoint": ([p, p, p], i32),
        "bmf_topk": ([p, p, i64, i32, p, p], i32),
        "bmf_topk_bf16": ([p, p, i64, i32, i32, p, p], i32),
        "bmf_topk_dev": ([p, p, i64, i32, i32, i32, p, p], i32),
        "bmf_topk_dev_noalloc": ([p, p, i64, i32, i32, i32, p, p], i32),
        "bmf_rmse_dev": ([p, p, p, p, i64, p], i32),
        "bmf_foldin": ([p, p, p, i32, i32, f32, f32, p, p], i32),
        "bmf_sgd_timing": ([p, p, p, i32], i32),
        "bmf_debug_wave_sum": ([p, p], i32),
        "bmf_chain_depth": ([i64, p, p, p], i32),
        "bmf_debug_chain_floor": ([i32, i32, p], i32),
        "bmf_debug_block_plan": ([i64, p, p, p, i32, i32, i32, i64, p, p], i32),
        "bmf_debug_topk_plan": ([i64, i32, i64, i32, i32, i32, p], i32),
        "bmf_stratum_order": ([i32, C.c_uint64, i32, i32, p], i32),
        "bmf_batch_create": ([i32, p, p, i32, p, pp], i32),
        "bmf_batch_destroy": ([p], None),
        "bmf_batch_last_error": ([p], C.c_char_p),
        "bmf_batch_set_option": ([p, i32, i64], i32),
        "bmf_batch_load": ([p, i32, p, p, p, i64], i32),
        "bmf_batch_tune": ([p], i32),
        "bmf_batch_epochs": ([p, i32, p], i32),
        "bmf_batch_problem": ([p, i32, pp], i32),
        "bmf_batch_info": ([p, i32, p, p, p], i32),
        "bmf_batch_timing": ([p, p, p, i32], i32),
        "bmf_server_create": ([p, p, pp], i32),
        "bmf_server_destroy": ([p], None),
        "bmf_server_last_error": ([p], C.c_char_p),
        "bmf_server_submit_topk": ([p, p, i32, i32, i32, p], i32),
        "bmf_server_submit_foldin": ([p, p, p, i32, i32, i32, p], i32),
        "bmf_server_poll": ([p, i64, i32, p, p, p, p, p, p], i32),
        "bmf_server_drain": ([p], i32),
        "bmf_server_get_stats": ([p, p, i32], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dptr(t) -> int:
    return None if t is None else C.c_void_p(t.data_ptr())


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Model:
    """One bmf context: m users, n items, k factors, b x b blocks."""

    def __init__(self, m: int, n: int, k: int, b: int, seed: Optional[int] = None,
                 order_mode: Optional[int] = None, order_seed: Optional[int] = None,
                 mu_mode: Optional[int] = None, sgd_kernel: Optional[int] = None,
                 waves: Optional[int] = None, out_of_core: Optional[bool] = None, _borrowed=None):
        self._owned = _borrowed is None
        if _borrowed is not None:
            self._h = _borrowed
            self.m, self.n, self.k, self.b = m, n, k, b
            return
        h = C.c_void_p()
        st = lib.bmf_create(m, n, k, b, C.byref(h))
        if st != 0:
            raise BmfError(st, lib.bmf_last_error(None).decode())
        self._h = h
        if waves is not None:
            self.set_option(OPT_WAVES_PER_BLOCK, waves)
        self.m, self.n, self.k, self.b = m, n, k, b
        if seed is not None:
            self.set_option(OPT_SEED, seed)
        if order_mode is not None:
            self.set_option(OPT_STRATUM_ORDER, order_mode)
        if order_seed is not None:
            self.set_option(OPT_ORDER_SEED, order_seed)
        if mu_mode is not None:
            self.set_option(OPT_MU_MODE, mu_mode)
        if sgd_kernel is not None:
            self.set_option(OPT_SGD_KERNEL, sgd_kernel)
        if out_of_core is not None:
            self.set_option(OPT_OUT_OF_CORE, int(bool(out_of_core)))

    # -- plumbing
    def _check(self, st: int):
        if st != 0:
            raise BmfError(st, lib.bmf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", True):
            lib.bmf_destroy(self._h)
        self._h = None

    destroy = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls (names follow bmf_*)
    def set_option(self, key: int, value: int):
        self._check(lib.bmf_set_option(self._h, key, int(value)))

    def synchronize(self):
        self._check(lib.bmf_synchronize(self._h))

    def load_ratings(self, u, i, r):
        u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
        self._check(lib.bmf_load_ratings(self._h, _ptr(u), _ptr(i), _ptr(r), u.shape[0]))

    def load_ratings_dev(self, u, i, r):
        self._check(lib.bmf_load_ratings_dev(self._h, _dptr(u), _dptr(i), _dptr(r), int(u.numel())))

    def epoch(self, lr: float, reg: float):
        self._check(lib.bmf_epoch(self._h, lr, reg))

    def epoch_hp(self, hp: Sequence[float]):
        hp = _c(hp, np.float32)
        self._check(lib.bmf_epoch_hp(self._h, _ptr(hp)))

    def fit(self, hp: Sequence[float], max_epochs: int, delta: float):
        """Epochs until the training RMSE improves by less than delta (see
        bmf_fit); returns (epochs run, final training RMSE)."""
        hp = _c(hp, np.float32)
        e = C.c_int32()
        r = C.c_double()
        self._check(lib.bmf_fit(self._h, _ptr(hp), int(max_epochs), float(delta), C.byref(e), C.byref(r)))
        return e.value, r.value

    def add_ratings(self, m_new: int, n_new: int, u, i, r, hp: Sequence[float], epochs_new: int):
        """Grow to m_new x n_new, train epochs_new epochs on the new ratings
        alone, then make all ratings the training set (see bmf_add_ratings)."""
        u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
        if not (u.shape == i.shape == r.shape):
            raise ValueError("u, i, r must have the same length")
        hp = _c(hp, np.float32)
        self._check(lib.bmf_add_ratings(self._h, int(m_new), int(n_new), _ptr(u), _ptr(i), _ptr(r),
                                        u.shape[0], _ptr(hp), int(epochs_new)))
        self.m, self.n = int(m_new), int(n_new)

    def plan_info(self, per_block: bool = False):
        """(kernel the next epoch runs, plan steps, LDS user slots), plus the
        steps of every block (b x b array) when per_block; see bmf_plan_info."""
        kern, steps, slots = C.c_int32(), C.c_int64(), C.c_int32()
        blocks = np.zeros((self.b, self.b), dtype=np.int64) if per_block else None
        self._check(lib.bmf_plan_info(self._h, C.byref(kern), C.byref(steps), C.byref(slots),
                                      _ptr(blocks) if per_block else None))
        out = (kern.value, steps.value, slots.value)
        return out + (blocks,) if per_block else out

    def epoch_count(self) -> int:
        out = C.c_int32()
        self._check(lib.bmf_epoch_count(self._h, C.byref(out)))
        return out.value

    def get_schedule(self, epoch: int) -> np.ndarray:
        out = np.zeros(self.b, dtype=np.int32)
        self._check(lib.bmf_get_schedule(self._h, epoch, _ptr(out)))
        return out

    def get_partition(self, nnz: int):
        bp = np.zeros(self.b * self.b + 1, dtype=np.int64)
        perm = np.zeros(nnz, dtype=np.int32)
        self._check(lib.bmf_get_partition(self._h, _ptr(bp), _ptr(perm)))
        return bp, perm

    def get_factors(self):
        P = np.zeros((self.m, self.k), dtype=np.float32)
        Q = np.zeros((self.n, self.k), dtype=np.float32)
        bu = np.zeros(self.m, dtype=np.float32)
        bi = np.zeros(self.n, dtype=np.float32)
        mu = C.c_double()
        self._check(lib.bmf_get_factors(self._h, _ptr(P), _ptr(Q), _ptr(bu), _ptr(bi), C.byref(mu)))
        return P, Q, bu, bi, mu.value

    def set_factors(self, P=None, Q=None, bu=None, bi=None, mu=None):
        args = [None if a is None else _c(a, np.float32) for a in (P, Q, bu, bi)]
        mu_c = None if mu is None else C.byref(C.c_double(float(mu)))
        self._check(lib.bmf_set_factors(self._h, *[_ptr(a) for a in args], mu_c))

    def factor_ptrs(self):
        ps = [C.c_void_p() for _ in range(4)]
        self._check(lib.bmf_factor_ptrs(self._h, *[C.byref(x) for x in ps]))
        return [x.value for x in ps]

    def rmse(self, u=None, i=None, r=None) -> float:
        out = C.c_double()
        if u is None:
            self._check(lib.bmf_rmse(self._h, None, None, None, 0, C.byref(out)))
        else:
            u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
            self._check(lib.bmf_rmse(self._h, _ptr(u), _ptr(i), _ptr(r), u.shape[0], C.byref(out)))
        return out.value

    def rmse_dev(self, u, i, r) -> float:
        """RMSE over device tensors (int32 u, i; float32 r) on the context's device."""
        out = C.c_double()
        self._check(lib.bmf_rmse_dev(self._h, _dptr(u), _dptr(i), _dptr(r), int(u.numel()), C.byref(out)))
        return out.value

    def loss(self, lr: float = 0.0, reg: float = 0.0, hp=None) -> float:
        hp = _c([lr, reg] * 4 if hp is None else hp, np.float32)
        out = C.c_double()
        self._check(lib.bmf_loss(self._h, _ptr(hp), C.byref(out)))
        return out.value

    def check_disjoint(self, pairing=None) -> int:
        """Race check of the strata on the device (bmf_check_disjoint): the
        count of ratings whose row another block of their stratum touches.
        pairing: None for the epochs' schedule, else int32 [b, b] block rows
        (pairing[s, j] = the row stratum s pairs with column j)."""
        out = C.c_int64()
        pr = None if pairing is None else _c(pairing, np.int32)
        if pr is not None and pr.size != self.b * self.b:
            raise ValueError("pairing must hold b * b block rows")
        self._check(lib.bmf_check_disjoint(self._h, _ptr(pr), C.byref(out)))
        return out.value

    def topk(self, users, K: int):
        users = _c(users, np.int32)
        items = np.zeros((users.shape[0], K), dtype=np.int32)
        scores = np.zeros((users.shape[0], K), dtype=np.float32)
        self._check(lib.bmf_topk(self._h, _ptr(users), users.shape[0], K, _ptr(items), _ptr(scores)))
        return items, scores

    def topk_bf16(self, users, K: int, Kc: int = 0):
        users = _c(users, np.int32)
        items = np.zeros((users.shape[0], K), dtype=np.int32)
        scores = np.zeros((users.shape[0], K), dtype=np.float32)
        self._check(lib.bmf_topk_bf16(self._h, _ptr(users), users.shape[0], K, Kc, _ptr(items), _ptr(scores)))
        return items, scores

    def topk_dev(self, users, K: int, precision: int, Kc: int, items_out, scores_out):
        self._check(lib.bmf_topk_dev(self._h, _dptr(users), int(users.numel()), K, precision, Kc,
                                     _dptr(items_out), _dptr(scores_out)))

    def topk_dev_noalloc(self, users, K: int, precision: int, Kc: int, items_out, scores_out):
        """topk_dev with the library's fixed device workspace (no device
        allocation; see bmf_topk_dev_noalloc)."""
        self._check(lib.bmf_topk_dev_noalloc(self._h, _dptr(users), int(users.numel()), K, precision, Kc,
                                             _dptr(items_out), _dptr(scores_out)))

    def foldin(self, items, r, passes: int, lr: float, reg: float):
        items, r = _c(items, np.int32), _c(r, np.float32)
        p = np.zeros(self.k, dtype=np.float32)
        bu = np.zeros(1, dtype=np.float32)
        self._check(lib.bmf_foldin(self._h, _ptr(items), _ptr(r), items.shape[0], passes, lr, reg, _ptr(p),
                                   _ptr(bu)))
        return p, float(bu[0])

    def sgd_timing(self, reset: bool = False):
        ms = C.c_double()
        launches = C.c_int64()
        self._check(lib.bmf_sgd_timing(self._h, C.byref(ms), C.byref(launches), int(reset)))
        return ms.value, launches.value


class Batch:
    """Many independent problems trained together (see bmf_batch_*): one
    launch per global stratum position runs that position's blocks of every
    problem that has one; successive positions follow in stream order."""

    def __init__(self, shapes, k: int, b=None, seed: Optional[int] = None, order_mode: Optional[int] = None,
                 order_seed: Optional[int] = None, waves: Optional[int] = None):
        m = np.array([s[0] for s in shapes], dtype=np.int64)
        n = np.array([s[1] for s in shapes], dtype=np.int64)
        bb = None if b is None else np.array(b, dtype=np.int32)
        h = C.c_void_p()
        st = lib.bmf_batch_create(len(shapes), _ptr(m), _ptr(n), k, _ptr(bb), C.byref(h))
        if st != 0:
            raise BmfError(st, "bmf_batch_create")
        self._h = h
        self.m, self.n, self.k = m, n, k
        for key, val in ((OPT_SEED, seed), (OPT_STRATUM_ORDER, order_mode), (OPT_ORDER_SEED, order_seed),
                         (OPT_WAVES_PER_BLOCK, waves)):
            if val is not None:
                self._check(lib.bmf_batch_set_option(self._h, key, int(val)))

    def _check(self, st: int):
        if st != 0:
            raise BmfError(st, lib.bmf_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.bmf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, p: int, u, i, r):
        u, i, r = _c(u, np.int32), _c(i, np.int32), _c(r, np.float32)
        self._check(lib.bmf_batch_load(self._h, p, _ptr(u), _ptr(i), _ptr(r), u.shape[0]))

    def tune(self):
        self._check(lib.bmf_batch_tune(self._h))

    def epochs(self, epochs: int, lr: float = None, reg: float = None, hp=None):
        hp = _c([lr, reg] * 4 if hp is None else hp, np.float32)
        self._check(lib.bmf_batch_epochs(self._h, epochs, _ptr(hp)))

    def problem(self, p: int) -> Model:
        h = C.c_void_p()
        self._check(lib.bmf_batch_problem(self._h, p, C.byref(h)))
        b, _, _ = self.info(p)
        return Model(int(self.m[p]), int(self.n[p]), self.k, b, _borrowed=h)

    def info(self, p: int):
        b, w, ms = C.c_int32(), C.c_int32(), C.c_double()
        self._check(lib.bmf_batch_info(self._h, p, C.byref(b), C.byref(w), C.byref(ms)))
        return b.value, w.value, ms.value

    def timing(self, reset: bool = False):
        ms, n = C.c_double(), C.c_int64()
        self._check(lib.bmf_batch_timing(self._h, C.byref(ms), C.byref(n), int(reset)))
        return ms.value, n.value


class ServerConfig(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("max_batches", C.c_int32), ("max_batch_rows", C.c_int32),
                ("max_requests_per_batch", C.c_int32), ("foldin_passes", C.c_int32), ("foldin_lr", C.c_float),
                ("foldin_reg", C.c_float), ("Kc", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("submitted", "completed", "rejected", "batches", "rows", "budget_bytes",
                                         "peak_bytes", "queue_depth")] + \
               [(f, C.c_double) for f in ("p50_ms", "p90_ms", "p99_ms", "max_ms", "mean_ms")]


class Server:
    """Continuous-batching server over a trained Model (see bmf_server_*)."""

    def __init__(self, model: Model, mem_budget_bytes: int = 0, max_batches: int = 0, max_batch_rows: int = 0,
                 max_requests_per_batch: int = 0, foldin_passes: int = 0, foldin_lr: float = 0.0,
                 foldin_reg: float = 0.0, Kc: int = 0):
        self.model = model
        cfg = ServerConfig(mem_budget_bytes, max_batches, max_batch_rows, max_requests_per_batch, foldin_passes,
                           foldin_lr, foldin_reg, Kc)
        h = C.c_void_p()
        st = lib.bmf_server_create(model._h, C.byref(cfg), C.byref(h))
        if st != 0:
            raise BmfError(st, lib.bmf_last_error(model._h).decode())
        self._h = h
        self._shape = {}

    def _check(self, st: int):
        if st != 0:
            raise BmfError(st, lib.bmf_server_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.bmf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_topk(self, users, K: int, precision: int = 1) -> int:
        users = _c(users, np.int32)
        rid = C.c_int64()
        self._check(lib.bmf_server_submit_topk(self._h, _ptr(users), users.shape[0], K, precision, C.byref(rid)))
        self._shape[rid.value] = (users.shape[0], K, False)
        return rid.value

    def submit_foldin(self, items, ratings, K: int, precision: int = 1) -> int:
        items, ratings = _c(items, np.int32), _c(ratings, np.float32)
        rid = C.c_int64()
        self._check(lib.bmf_server_submit_foldin(self._h, _ptr(items), _ptr(ratings), items.shape[0], K, precision,
                                                 C.byref(rid)))
        self._shape[rid.value] = (1, K, True)
        return rid.value

    def poll(self, rid: int, wait: bool = True):
        rows, K, fold = self._shape[rid]
        done = C.c_int32()
        items = np.zeros((rows, K), dtype=np.int32)
        scores = np.zeros((rows, K), dtype=np.float32)
        p = np.zeros(self.model.k, dtype=np.float32) if fold else None
        bu = np.zeros(1, dtype=np.float32) if fold else None
        lat = C.c_int64()
        self._check(lib.bmf_server_poll(self._h, rid, int(wait), C.byref(done), _ptr(items), _ptr(scores), _ptr(p),
                                        _ptr(bu), C.byref(lat)))
        if not done.value:
            return None
        del self._shape[rid]
        out = {"items": items, "scores": scores, "latency_ms": lat.value / 1e6}
        if fold:
            out["p"] = p
            out["bu"] = float(bu[0])
        return out

    def drain(self):
        self._check(lib.bmf_server_drain(self._h))

    def stats(self, reset: bool = False) -> dict:
        st = ServerStats()
        self._check(lib.bmf_server_get_stats(self._h, C.byref(st), int(reset)))
        return {f: getattr(st, f) for f, _ in st._fields_}


def stratum_order(b: int, seed: int, epoch: int, mode: int) -> np.ndarray:
    out = np.zeros(b, dtype=np.int32)
    st = lib.bmf_stratum_order(b, seed, epoch, mode, _ptr(out))
    if st != 0:
        raise BmfError(st, "bmf_stratum_order")
    return out


PLAN_FIRST = 1 << 30
PLAN_LAST = 1 << 31


def block_plan(u_local, i_local, r, cb: int, slots: int, chunk: int) -> np.ndarray:
    """Step plan of one block (host only): uint32 array (steps, 4, 4) of
    {meta, rating bits, u_local, index} records (see bmf_debug_block_plan)."""
    u_local = _c(u_local, np.int32)
    i_local = _c(i_local, np.int32)
    r = _c(r, np.float32)
    n = len(u_local)
    ns = np.zeros(1, dtype=np.int64)
    st = lib.bmf_debug_block_plan(n, _ptr(u_local), _ptr(i_local), _ptr(r), cb, slots, chunk, 0, _ptr(ns), None)
    if st != 0:
        raise BmfError(st, lib.bmf_last_error(None).decode())
    out = np.zeros((int(ns[0]), 4, 4), dtype=np.uint32)
    st = lib.bmf_debug_block_plan(n, _ptr(u_local), _ptr(i_local), _ptr(r), cb, slots, chunk, int(ns[0]), _ptr(ns),
                                  _ptr(out))
    if st != 0:
        raise BmfError(st, lib.bmf_last_error(None).decode())
    return out


def topk_plan(n: int, k: int, nu: int, K: int, precision: int = 0, Kc: int = 0) -> dict:
    """The plan a top-K request gets (see bmf_debug_topk_plan; host only)."""
    out = np.zeros(7, dtype=np.int64)
    st = lib.bmf_debug_topk_plan(n, k, nu, K, precision, Kc, _ptr(out))
    if st != 0:
        raise BmfError(st, "bmf_debug_topk_plan")
    keys = ("samples", "rank", "capacity", "need", "splits", "per_split", "workspace_bytes")
    return {key: int(v) for key, v in zip(keys, out)}


def chain_depth(u, i) -> int:
    """Dependency depth of a block's ratings in processing order (see
    bmf_chain_depth; host only)."""
    u, i = _c(u, np.int32), _c(i, np.int32)
    out = np.zeros(1, dtype=np.int64)
    st = lib.bmf_chain_depth(u.shape[0], _ptr(u), _ptr(i), _ptr(out))
    if st != 0:
        raise BmfError(st, "bmf_chain_depth")
    return int(out[0])


def chain_floor_ns(k: int, steps: int = 1 << 18) -> float:
    """GPU time per dependent step of the planned SGD kernel's step code
    (see bmf_debug_chain_floor)."""
    out = np.zeros(1, dtype=np.float64)
    st = lib.bmf_debug_chain_floor(k, steps, _ptr(out))
    if st != 0:
        raise BmfError(st, lib.bmf_last_error(None).decode())
    return float(out[0])


def debug_wave_sum(x) -> np.ndarray:
    x = _c(x, np.float32)
    out = np.zeros(256, dtype=np.float32)
    st = lib.bmf_debug_wave_sum(_ptr(x), _ptr(out))
    if st != 0:
        raise BmfError(st, lib.bmf_last_error(None).decode())
    return out.reshape(4, 64)
