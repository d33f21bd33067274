"""The C ABI: the built library exports every symbol the header declares,
and the host-only logic (argument checks, stratum order) behaves as
documented.  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmf.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bmf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    from paper_1907_07410_amd import binding
    return binding


def test_header_declares_the_core_calls():
    syms = declared_symbols()
    for name in ["bmf_create", "bmf_load_ratings", "bmf_epoch", "bmf_rmse", "bmf_topk", "bmf_topk_bf16",
                 "bmf_foldin", "bmf_get_partition", "bmf_get_schedule", "bmf_destroy", "bmf_last_error"]:
        assert name in syms


def test_library_exports_every_declared_symbol(binding):
    lib = C.CDLL(binding.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert missing == []


def test_binding_constants_match_the_header(binding):
    """The binding's option keys and status codes carry the header's values."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    opts = dict(re.findall(r"\bBMF_OPT_([A-Z_]+)\s*=\s*(\d+)", text))
    codes = dict(re.findall(r"\bBMF_(OK|E_[A-Z]+)\s*=\s*(-?\d+)", text))
    assert len(opts) == 10 and len(codes) == 6
    for name, value in opts.items():
        assert getattr(binding, "OPT_" + name) == int(value), name
    for name, value in codes.items():
        assert getattr(binding, "BMF_" + name) == int(value), name


def test_create_rejects_bad_sizes_without_touching_the_device(binding):
    h = C.c_void_p()
    for args in [(0, 5, 4, 2), (5, 0, 4, 2), (5, 5, 0, 2), (5, 5, 4, 0), (5, 5, 2000, 2), (5, 5, 4, 10**5)]:
        st = binding.lib.bmf_create(*args, C.byref(h))
        assert st == binding.BMF_E_INVAL
        assert h.value is None
        assert binding.lib.bmf_last_error(None)
        assert binding.lib.bmf_server_last_error(None) == b""
    assert binding.lib.bmf_create(5, 5, 4, 2, None) == binding.BMF_E_INVAL


def test_null_context_is_rejected(binding):
    assert binding.lib.bmf_epoch(None, 0.1, 0.1) == binding.BMF_E_INVAL
    assert binding.lib.bmf_rmse(None, None, None, None, 0, None) == binding.BMF_E_INVAL
    binding.lib.bmf_destroy(None)


@pytest.mark.parametrize("b", [1, 2, 5, 64, 128, 3072])
def test_stratum_order_matches_oracle(binding, orc, b):
    for mode in (0, 1):
        for e in (0, 1, 7, 123):
            got = binding.stratum_order(b, 2001, e, mode)
            assert np.array_equal(got, orc.schedule(b, 2001, e, mode))


def test_stratum_order_argument_checks(binding):
    out = np.zeros(4, dtype=np.int32)
    p = out.ctypes.data_as(C.c_void_p)
    assert binding.lib.bmf_stratum_order(0, 1, 0, 0, p) == binding.BMF_E_INVAL
    assert binding.lib.bmf_stratum_order(4, 1, -1, 0, p) == binding.BMF_E_INVAL
    assert binding.lib.bmf_stratum_order(4, 1, 0, 2, p) == binding.BMF_E_INVAL
    assert binding.lib.bmf_stratum_order(4, 1, 0, 0, None) == binding.BMF_E_INVAL
