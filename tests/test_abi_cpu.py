"""The C-ABI library loads on the host and exports every entry point of include/rtcc.h (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtcc.h")


def _lib():
    import paper_2205_05175_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("librtcc.so not built")
    return P, P.load_library()


def test_header_symbols_exported():
    P, L = _lib()
    decl = set(re.findall(r"\b(rtcc_[a-z0-9_]+)\s*\(", open(HEADER).read()))
    assert decl == set(P.EXPORTED)
    for name in decl:
        assert hasattr(L, name), name


def test_init_rejects_invalid_arguments_without_gpu_work():
    P, L = _lib()
    ctx = ctypes.c_void_p()
    a = np.zeros(16)
    dp = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.rtcc_init(ctypes.byref(ctx), 0, 1, dp, dp, dp, 0, None) == -1
    assert b"invalid" in L.rtcc_last_error(None)
    assert L.rtcc_init(ctypes.byref(ctx), 1, 1, None, dp, dp, 0, None) == -1
    assert L.rtcc_init(ctypes.byref(ctx), 1, 1, dp, dp, dp, 7, None) == -1
    assert L.rtcc_init(None, 1, 1, dp, dp, dp, 0, None) == -1
    assert not ctx.value


def test_null_context_calls_fail_cleanly():
    _, L = _lib()
    assert L.rtcc_set_precision(None, 0) == -1
    assert L.rtcc_info(None, None) == -1
    L.rtcc_destroy(None)
