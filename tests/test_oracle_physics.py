"""Physics pins of the oracle (no GPU): exactness for two electrons, stationarity, Lagrangian structure."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bruteforce, ccsd, field, ground, integrators, spinorb
from synth import make_system, pack_state, random_state, unpack_state


def _ground(o, v, seed=0):
    eri, fock, mu = make_system(o, v, seed=seed)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    t1, t2, l1, l2, e = ground.solve(S, fock)
    return S, (t1, t2, l1, l2), e


def test_two_electron_ccsd_is_fci():
    """For two electrons CCSD is exact: E_ref + E_CCSD is the lowest FCI eigenvalue (singlet)."""
    o, v = 1, 4
    S, amps, e = _ground(o, v)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    dim = bf.space.dim
    H = np.column_stack([bruteforce._apply_hamiltonian(bf.space, bf.h, bf.g, np.eye(dim)[:, k].astype(complex))
                         for k in range(dim)])
    w, U = np.linalg.eigh(H)
    ref = bf.space.ref
    # ground state = lowest eigenvector with weight on the closed-shell reference
    k = next(k for k in range(dim) if abs(U[ref, k]) > 0.1)
    e0 = H[ref, ref].real
    assert abs((e0 + e.real) - w[k]) < 1e-10


def test_zero_field_stationarity():
    """At the converged ground state and zero field both time derivatives vanish."""
    S, amps, _ = _ground(3, 6)
    d = ccsd.rhs(S, *amps, np.zeros(3))
    assert max(np.max(np.abs(x)) for x in d) < 1e-11


def test_lambda_residual_is_lagrangian_gradient():
    """R_L = dL/dt for L = E(T) + sum lambda R_T(T) (directional derivative, exact 5-point stencil)."""
    o, v = 2, 4
    eri, fock, mu = make_system(o, v, seed=3)
    S = ccsd.SpinOrbitalSystem(eri, fock + 0.05 * np.ones_like(fock), mu, o, v)
    t1, t2, l1, l2 = random_state(o, v, 11, 0.1, 0.05)
    T1, T2 = spinorb.cs_to_so(t1, t2)
    L1, L2 = spinorb.cs_to_so(l1, l2)
    d1, d2, _, _ = random_state(o, v, 12, 1.0, 1.0)
    D1, D2 = spinorb.cs_to_so(d1, d2)
    L = lambda s: ccsd.lagrangian(S.f0, S.g, T1 + s * D1, T2 + s * D2, L1, L2)
    h = 1e-2
    dL = (L(-2 * h) - 8 * L(-h) + 8 * L(h) - L(2 * h)) / (12 * h)
    R1, R2 = ccsd.l_residual(S.f0, S.g, T1, T2, L1, L2)
    pred = np.sum(R1 * D1) + 0.25 * np.sum(R2 * D2)
    assert abs(dL - pred) < 1e-10 * max(1.0, abs(pred))


def test_t_residual_is_lagrangian_lambda_gradient():
    """dL/dlambda = R_T: the Lagrangian is linear in Lambda."""
    o, v = 2, 3
    eri, fock, mu = make_system(o, v, seed=4)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    t1, t2, l1, l2 = random_state(o, v, 13, 0.1, 0.05)
    d1, d2, _, _ = random_state(o, v, 14, 1.0, 1.0)
    T1, T2 = spinorb.cs_to_so(t1, t2)
    L1, L2 = spinorb.cs_to_so(l1, l2)
    D1, D2 = spinorb.cs_to_so(d1, d2)
    dL = (ccsd.lagrangian(S.f0, S.g, T1, T2, L1 + D1, L2 + D2)
          - ccsd.lagrangian(S.f0, S.g, T1, T2, L1, L2))
    R1, R2 = ccsd.t_residual(S.f0, S.g, T1, T2)
    assert abs(dL - (np.sum(R1 * D1) + 0.25 * np.sum(R2 * D2))) < 1e-12


def _propagate(S, y, h, nsteps, Efun):
    o, v = S.o, S.v
    f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, o, v), Efun(t)))
    ys = [y]
    for k in range(nsteps):
        y = integrators.rk4_step(f, k * h, y, h)
        ys.append(y)
    return ys


def test_two_electron_delta_kick_dynamics_matches_fci():
    """RT-CCSD after a delta kick reproduces exact TD-FCI <mu_z>(t) for two electrons (RK4 error ~h^4)."""
    o, v = 1, 3
    S, amps, _ = _ground(o, v)
    kappa, n = 2e-2, np.array([0.0, 0.0, 1.0])
    kicked = field.kick(S, amps, kappa, n)
    # exact: Psi(0+) = exp(i kappa mu_z) Psi0, then exp(-i H t)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    dim = bf.space.dim
    cols = lambda A1, A2: np.column_stack([bruteforce._apply_hamiltonian(bf.space, A1, A2, np.eye(dim)[:, k].astype(complex))
                                           for k in range(dim)])
    H = cols(bf.h, bf.g)
    M = cols(S.mu[2], None)
    w, U = np.linalg.eigh(H)
    k0 = next(k for k in range(dim) if abs(U[bf.space.ref, k]) > 0.1)
    psi = sla.expm(1j * kappa * M) @ U[:, k0]
    T = 2.0
    exact = []
    for nsteps in (20, 40):
        h = T / nsteps
        psit = sla.expm(-1j * H * T) @ psi
        exact = (np.vdot(psit, M @ psit) / np.vdot(psit, psit)).real
        ys = _propagate(S, pack_state(*kicked), h, nsteps, lambda t: np.zeros(3))
        mu_cc = ccsd.dipole(S, *unpack_state(ys[-1], o, v))[2]
        exact_list = exact
        if nsteps == 20:
            e20 = abs(mu_cc.real - exact_list)
        else:
            e40 = abs(mu_cc.real - exact_list)
    assert e40 < 1e-6
    assert 8 < e20 / e40 < 24  # fourth order
    # the kick itself: mu(0+) equals <Psi(0+)|mu|Psi(0+)> exactly (up to the 100-substep RK4 error)
    mu0 = ccsd.dipole(S, *kicked)[2]
    assert abs(mu0 - np.vdot(psi, M @ psi)) < 1e-11


def _two_electron_kick_case():
    o, v = 1, 3
    S, amps, _ = _ground(o, v)
    kappa, n = 2e-2, np.array([0.0, 0.0, 1.0])
    kicked = field.kick(S, amps, kappa, n)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    dim = bf.space.dim
    cols = lambda A1, A2: np.column_stack([bruteforce._apply_hamiltonian(bf.space, A1, A2, np.eye(dim)[:, k].astype(complex))
                                           for k in range(dim)])
    H = cols(bf.h, bf.g)
    M = cols(S.mu[2], None)
    w, U = np.linalg.eigh(H)
    k0 = next(k for k in range(dim) if abs(U[bf.space.ref, k]) > 0.1)
    psi = sla.expm(1j * kappa * M) @ U[:, k0]

    def exact(T):
        psit = sla.expm(-1j * H * T) @ psi
        return (np.vdot(psit, M @ psit) / np.vdot(psit, psit)).real

    f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, o, v), np.zeros(3)))
    mu_z = lambda y: ccsd.dipole(S, *unpack_state(y, o, v))[2].real
    return pack_state(*kicked), f, mu_z, exact


def test_two_electron_gauss_legendre_matches_fci():
    """Implicit two-stage Gauss-Legendre on the kicked two-electron system: TD-FCI <mu_z>(T) with
    the fourth-order error ratio when h is halved."""
    y0, f, mu_z, exact = _two_electron_kick_case()
    c, A, b = integrators.gauss_legendre_tableau(2)
    T = 2.0
    errs = []
    for nsteps in (10, 20):
        h, y = T / nsteps, y0
        for k in range(nsteps):
            y, it = integrators.implicit_rk_step(f, k * h, y, h, c, A, b, 1e-14, 100)
        errs.append(abs(mu_z(y) - exact(T)))
    assert errs[1] < 1e-6
    assert 8 < errs[0] / errs[1] < 24


def test_two_electron_rkf45_matches_fci():
    """Adaptive Fehlberg 4(5) on the same system: accepted samples follow TD-FCI to within the
    accumulated tolerance."""
    y0, f, mu_z, exact = _two_electron_kick_case()
    samples = []
    y, t, nacc, nrej, _ = integrators.embedded_propagate(
        f, 0.0, y0, 0.05, 1e-9, 3.0, integrators.RKF45_C, integrators.RKF45_A, integrators.RKF45_B4,
        integrators.RKF45_B5, 4, on_accept=lambda tt, yy: samples.append((tt, mu_z(yy))))
    assert t == 3.0 and nacc >= 5
    assert max(abs(m - exact(tt)) for tt, m in samples) < 20 * nacc * 1e-9


def test_lagrangian_conserved_field_free():
    """Field-free propagation conserves L = <0|(1+Lambda)Hbar|0>; RK4 drift falls as h^4."""
    o, v = 2, 4
    S, amps, _ = _ground(o, v)
    kicked = field.kick(S, amps, 0.05, np.array([1.0, 0.0, 0.0]))
    drifts = []
    for nsteps in (10, 20):
        ys = _propagate(S, pack_state(*kicked), 1.0 / nsteps, nsteps, lambda t: np.zeros(3))
        Ls = []
        for y in (ys[0], ys[-1]):
            a = unpack_state(y, o, v)
            T1, T2 = spinorb.cs_to_so(a[0], a[1])
            L1, L2 = spinorb.cs_to_so(a[2], a[3])
            Ls.append(ccsd.lagrangian(S.f0, S.g, T1, T2, L1, L2))
        drifts.append(abs(Ls[1] - Ls[0]))
    assert drifts[1] < 1e-6
    assert drifts[0] / drifts[1] > 8


def test_linear_response_scaling():
    """The induced dipole after a weak kick scales linearly with the kick strength."""
    o, v = 2, 4
    S, amps, _ = _ground(o, v)
    mu_gs = ccsd.dipole(S, *amps)[2].real
    ind = []
    for kappa in (1e-3, 5e-4):
        kicked = field.kick(S, amps, kappa, np.array([0.0, 0.0, 1.0]))
        ys = _propagate(S, pack_state(*kicked), 0.05, 20, lambda t: np.zeros(3))
        ind.append((ccsd.dipole(S, *unpack_state(ys[-1], o, v))[2].real - mu_gs) / kappa)
    assert abs(ind[0] - ind[1]) < 2e-3 * abs(ind[1]) + 1e-9


def _strong_field_case():
    """(2,4) ground state in a strong Gaussian pulse: E0 = 100 au, sigma = 0.05 au, centre 0.25 au."""
    o, v = 2, 4
    S, amps, _ = _ground(o, v)
    y0 = pack_state(*amps)
    E0, sig, nu = 100.0, 0.05, 0.25
    f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, o, v),
                                           field.gaussian(t, E0, 0.0, sig, nu, [0, 0, 1])))
    t2norm = lambda yy: float(np.linalg.norm(unpack_state(yy, o, v)[1]))
    return f, y0, t2norm, (nu - 5 * sig, nu + 5 * sig)


def test_strong_field_rk4_diverges_and_mixed_step_is_stable():
    """Paper (Results, strong fields): RK4 with h = 0.01 au diverges in a 100 au pulse, while small steps
    during the pulse (h1) and the usual h2 after it give a bounded |T2|."""
    f, y0, t2norm, on = _strong_field_case()
    y, norms = y0.copy(), []
    with np.errstate(all="ignore"):
        for k in range(50):
            y = integrators.rk4_step(f, 0.01 * k, y, 0.01)
            norms.append(t2norm(y))
            if not np.isfinite(norms[-1]) or norms[-1] > 1e6:
                break
    assert not (np.isfinite(norms[-1]) and norms[-1] <= 1e6), "plain RK4 at h = 0.01 should diverge"
    plan = integrators.mixed_step_plan(0.0, 0.6, 1e-3, 0.01, on)
    assert abs(sum(h for _, h in plan) - 0.6) < 1e-12
    assert all(abs(h - 1e-3) < 1e-15 for t, h in plan if on[0] <= t < on[1] - 1e-3)
    norms = []
    integrators.rk4_propagate_plan(f, y0, plan, lambda k, t, yy: norms.append(t2norm(yy)))
    assert np.all(np.isfinite(norms)) and max(norms) < 1e3
