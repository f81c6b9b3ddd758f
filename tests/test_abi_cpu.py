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


def test_builtin_tableaux_match_oracle():
    """The library's tableaux (host-only call) against the oracle's: RK4 and the corrected Cash-Karp and
    Fehlberg pairs exactly as published, Gauss-Legendre against the oracle's collocation construction."""
    from oracle import integrators as I
    P, L = _lib()

    def dense(A, s):
        return np.array([[float(A[i][j]) if j < len(A[i]) else 0.0 for j in range(s)] for i in range(s)])

    cases = {
        "rk4": (dense(I.RK4_A, 4), I.RK4_B, I.RK4_C, [0.0] * 4, 0),
        "cashkarp": (dense(I.CK_A, 6), I.CK_B5, I.CK_C, I.CK_B4, 4),
        "rkf45": (dense(I.RKF45_A, 6), I.RKF45_B4, I.RKF45_C, I.RKF45_B5, 4),
    }
    for name, (A, b, c, be, p) in cases.items():
        T = P.Tableau.builtin(name)
        TA, Tb, Tc, Tbe = T.arrays()
        assert T.err_order == p
        assert np.array_equal(TA, A), name
        assert np.array_equal(Tb, np.array([float(x) for x in b]))
        assert np.array_equal(Tc, np.array([float(x) for x in c]))
        assert np.array_equal(Tbe, np.array([float(x) for x in be]))
    for name, s in (("gl2", 2), ("gl3", 3)):
        T = P.Tableau.builtin(name)
        TA, Tb, Tc, _ = T.arrays()
        c, A, b = I.gauss_legendre_tableau(s)
        assert T.err_order == 0 and T.stages == s
        assert np.allclose(TA, A, atol=4e-15, rtol=0) and np.allclose(Tb, b, atol=4e-15, rtol=0)
        assert np.allclose(Tc, c, atol=1e-15, rtol=0)
    with pytest.raises(P.RTCCError):
        P.Tableau.builtin(99)
    assert L.rtcc_tableau_builtin(1, None) == -1


def test_peak_probe_rejects_bad_arguments():
    """rtcc_peak_probe validates its arguments before touching a device: an unknown kind, an empty size and a
    null output return RTCC_EINVAL."""
    import ctypes
    P, L = _lib()
    v = ctypes.c_double(0.0)
    assert L.rtcc_peak_probe(4, 100, ctypes.byref(v)) == -1
    assert L.rtcc_peak_probe(-1, 100, ctypes.byref(v)) == -1
    assert L.rtcc_peak_probe(2, 0, ctypes.byref(v)) == -1
    assert L.rtcc_peak_probe(2, 100, None) == -1
    assert b"invalid" in L.rtcc_last_error(None)
    with pytest.raises(KeyError):
        P.peak_probe("fp16", 10)
