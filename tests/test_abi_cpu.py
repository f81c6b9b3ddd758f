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


def test_mixed_schedule_matches_oracle_plan():
    """rtcc_mixed_schedule is host-only: compare it with the oracle's mixed step-size plan."""
    P, L = _lib()
    from oracle import integrators
    cases = [(0.0, 0.6, 1e-3, 0.01, P.Field.gaussian(100.0, 0.0, 0.05, 0.25, [0, 0, 1])),
             (0.0, 2.0, 1e-4, 0.02, P.Field.gaussian(1.0, 0.5, 1e-4, 5e-4, [0, 0, 1])),
             (1.0, 3.05, 0.01, 0.02, P.Field.gaussian(1.0, 0.5, 0.1, 0.5, [1, 0, 0])),  # pulse over before t0
             (0.0, 1.0, 0.01, 0.03, P.Field.none())]
    for t0, t1, h1, h2, f in cases:
        got = P.mixed_schedule(t0, t1, h1, h2, f)
        on = (f.t0 - 5 * f.sigma, f.t0 + 5 * f.sigma) if f.kind == 1 else None
        plan = integrators.mixed_step_plan(t0, t1, h1, h2, on)
        ref = np.array([t0] + [t + h for t, h in plan])
        assert got.size == ref.size and np.max(np.abs(got - ref)) < 1e-12
    n = ctypes.c_int(0)
    assert L.rtcc_mixed_schedule(0.0, 1.0, -1.0, 0.01, None, 0, None, ctypes.byref(n)) == -1
    short = np.zeros(3)
    assert L.rtcc_mixed_schedule(0.0, 1.0, 0.1, 0.1, None, 3, short.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(n)) == -1
