"""General Runge-Kutta tableaux on the GPU (rtcc_step_tableau, rtcc_propagate_embedded) against the oracle.

Cases start from a seeded random non-stationary state (synth.random_state) of a (3,6) system in a
Gaussian pulse, so the oracle evaluates the same right-hand sides in seconds:
* the RK4 tableau through the general engine is bitwise rtcc_step_rk4 (same kernels, same coefficients);
* one Cash-Karp and one Fehlberg step: the state and the embedded error estimate equal the oracle's;
* the general adaptive driver with the Cash-Karp tableau is bitwise rtcc_propagate_cashkarp, and with
  Fehlberg's pair reproduces the oracle's whole propagation (same trials, times, dipoles);
* implicit Gauss-Legendre steps (two and three stages): the state and the number of fixed-point sweeps
  equal the oracle's in FP64; in FP32 the state agrees to single-precision accuracy;
* an implicit step that cannot converge in max_iter sweeps returns RTCC_ENOTCONV and leaves y alone.
"""
import numpy as np
import pytest

from synth import make_system, pack_state, random_state, unpack_state

pytestmark = pytest.mark.gpu

O, V = 3, 6
PULSE = dict(E0=0.05, omega=0.4, sigma=0.3, t0=0.5, n=(0.3, -0.2, 1.0))


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _oracle():
    from oracle import ccsd, field
    eri, fock, mu = make_system(O, V, 1)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, O, V)
    p = PULSE

    def f(t, y):
        E = field.gaussian(t, p["E0"], p["omega"], p["sigma"], p["t0"], p["n"])
        return pack_state(*ccsd.rhs(S, *unpack_state(y, O, V), E))

    return S, f


def _gpu(prec="fp64"):
    from paper_2205_05175_amd import RTCC, Field
    R = RTCC(*make_system(O, V, 1), O, V, prec)
    p = PULSE
    return R, Field.gaussian(p["E0"], p["omega"], p["sigma"], p["t0"], p["n"])


def _y0():
    return pack_state(*random_state(O, V, 21, 0.05, 0.02))


def _dev(y):
    import torch
    return torch.tensor(y, dtype=torch.complex128, device="cuda")


def test_rk4_tableau_is_step_rk4():
    import torch
    print("tableau rk4 == rtcc_step_rk4 (3,6) fp64 and bf16x3", flush=True)
    for prec in ("fp64", "bf16x3"):
        R, fld = _gpu(prec)
        a, b = _dev(_y0()), _dev(_y0())
        R.step_rk4(a, 0.3, 0.05, fld)
        dl, sw = R.step_tableau(b, 0.3, 0.05, "rk4", fld)
        torch.cuda.synchronize()
        assert dl is None and sw == 1
        assert torch.equal(a, b), prec
        R.close()


@pytest.mark.parametrize("name", ["cashkarp", "rkf45"])
def test_embedded_step_matches_oracle(name):
    from oracle import integrators as I
    print(f"tableau {name} one step (3,6) fp64", flush=True)
    S, f = _oracle()
    y0 = _y0()
    h, t = 0.08, 0.2
    if name == "cashkarp":
        c, A, badv, bemb = I.CK_C, I.CK_A, I.CK_B5, I.CK_B4
    else:
        c, A, badv, bemb = I.RKF45_C, I.RKF45_A, I.RKF45_B4, I.RKF45_B5
    yref, dref = I.embedded_trial(f, t, y0, h, c, A, badv, bemb)
    R, fld = _gpu()
    y = _dev(y0)
    dl, _ = R.step_tableau(y, t, h, name, fld)
    got = y.cpu().numpy()
    assert np.abs(got - yref).max() < 1e-12 * max(1.0, np.abs(yref).max())
    assert abs(dl - dref) < 1e-9 * dref + 1e-15
    R.close()


def test_embedded_driver_is_cashkarp_driver():
    import torch
    print("propagate_embedded(cashkarp) == propagate_cashkarp (3,6) fp64", flush=True)
    R, fld = _gpu()
    a, b = _dev(_y0()), _dev(_y0())
    ra = R.propagate_cashkarp(a, 0.0, 1.5, 0.1, 1e-8, fld)
    rb = R.propagate_embedded(b, 0.0, 1.5, 0.1, 1e-8, "cashkarp", fld)
    torch.cuda.synchronize()
    assert ra[2:] == rb[2:]
    assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])
    assert torch.equal(a, b)
    R.close()


def test_rkf45_propagation_matches_oracle():
    import torch
    from oracle import ccsd, integrators as I
    print("propagate_embedded(rkf45) (3,6) fp64 eps=1e-8 vs oracle", flush=True)
    S, f = _oracle()
    y0 = _y0()
    ref = []
    yr, tr, nacc, nrej, hn = I.embedded_propagate(
        f, 0.0, y0, 0.1, 1e-8, 1.5, I.RKF45_C, I.RKF45_A, I.RKF45_B4, I.RKF45_B5, 4,
        on_accept=lambda t, y: ref.append((t, ccsd.dipole(S, *unpack_state(y, O, V)))))
    R, fld = _gpu()
    y = _dev(y0)
    ts, mus, na, nr, hg = R.propagate_embedded(y, 0.0, 1.5, 0.1, 1e-8, "rkf45", fld)
    torch.cuda.synchronize()
    print(f"  oracle {nacc} accepted {nrej} rejected; gpu {na} / {nr}", flush=True)
    assert (na, nr) == (nacc, nrej) and nrej >= 1
    assert np.abs(ts - np.array([t for t, _ in ref])).max() < 1e-10 and ts[-1] == 1.5
    assert np.abs(mus - np.array([m for _, m in ref])).max() < 1e-10
    assert np.abs(y.cpu().numpy() - yr).max() < 1e-10
    assert abs(hg - hn) < 1e-8 * hn
    R.close()


@pytest.mark.parametrize("name,s", [("gl2", 2), ("gl3", 3)])
def test_gauss_legendre_step_matches_oracle(name, s):
    from oracle import integrators as I
    print(f"implicit {name} step (3,6) fp64 / fp32 vs oracle", flush=True)
    S, f = _oracle()
    y0 = _y0()
    h, t, tol = 0.05, 0.4, 1e-12
    c, A, b = I.gauss_legendre_tableau(s)
    yref, sweeps = I.implicit_rk_step(f, t, y0, h, c, A, b, tol, 100)
    R, fld = _gpu()
    y = _dev(y0)
    dl, sw = R.step_tableau(y, t, h, name, fld, tol=tol, max_iter=100)
    print(f"  oracle {sweeps} sweeps, gpu {sw}", flush=True)
    assert dl is None and sw == sweeps and sweeps >= 3
    assert np.abs(y.cpu().numpy() - yref).max() < 1e-11 * max(1.0, np.abs(yref).max())
    R.close()
    # complex FP32 contractions: converged to a tolerance above FP32 rounding
    R, fld = _gpu("fp32")
    y = _dev(y0)
    # (the sweep-to-sweep change of h k cannot fall below h |k| times the FP32 rounding, ~5e-9 here)
    _, sw32 = R.step_tableau(y, t, h, name, fld, tol=1e-7, max_iter=100)
    err = np.abs(y.cpu().numpy() - yref).max()
    print(f"  fp32: {sw32} sweeps, max |dy| = {err:.2e}", flush=True)
    assert err < 2e-6
    R.close()


def test_implicit_step_not_converged_leaves_state():
    import torch
    from paper_2205_05175_amd import RTCCError
    print("implicit gl2 max_iter=1: RTCC_ENOTCONV (3,6) fp64", flush=True)
    R, fld = _gpu()
    y = _dev(_y0())
    y_before = y.clone()
    with pytest.raises(RTCCError) as e:
        R.step_tableau(y, 0.0, 0.05, "gl2", fld, tol=1e-14, max_iter=1)
    assert e.value.code == -5
    torch.cuda.synchronize()
    assert torch.equal(y, y_before)
    # a tableau the engine refuses: implicit with more than three stages
    from paper_2205_05175_amd import Tableau
    bad = Tableau.from_arrays(np.full((4, 4), 0.25), [0.25] * 4, [1.0] * 4)
    with pytest.raises(RTCCError):
        R.step_tableau(y, 0.0, 0.05, bad, fld)
    R.close()
