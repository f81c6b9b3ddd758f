"""The factorised oracle against the brute-force determinant-space definitions.

Pins (no GPU): at random NON-stationary complex amplitudes and a random
non-diagonal symmetric Fock matrix, the factorised spin-orbital equations
must equal the definitions of Eq. derivT (T residual), Eq. derivL (Lambda
residual in commutator form), Eq. dipole and <0|Hbar|0>, evaluated with
explicit second-quantised operators on the full determinant space.
"""
import numpy as np
import pytest

from oracle import bruteforce, ccsd, spinorb
from synth import make_system, random_state, random_symmetric

CASES = [(1, 3), (2, 3), (2, 4), (3, 3)]


def _setup(o, v, seed, fov=True):
    eri, fock, mu = make_system(o, v, seed=seed)
    rng = np.random.default_rng(100 + seed)
    pert = random_symmetric(o + v, 0.1, rng)
    if not fov:
        pert[:o, o:] = 0.0
        pert[o:, :o] = 0.0
    fock = fock + pert
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    t1, t2, l1, l2 = random_state(o, v, seed + 7, 0.1, 0.05)
    T1, T2 = spinorb.cs_to_so(t1, t2)
    L1, L2 = spinorb.cs_to_so(l1, l2)
    return S, (t1, t2, l1, l2), (T1, T2, L1, L2)


@pytest.mark.parametrize("o,v", CASES)
def test_t_residual_and_energy(o, v):
    S, _, (T1, T2, _, _) = _setup(o, v, 1)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    R1b, R2b, Eb = bf.t_residual(T1, T2)
    R1, R2 = ccsd.t_residual(S.f0, S.g, T1, T2)
    assert np.max(np.abs(R1b)) > 1e-2 and np.max(np.abs(R2b)) > 1e-2  # far from stationary
    assert np.max(np.abs(R1 - R1b)) < 1e-12
    assert np.max(np.abs(R2 - R2b)) < 1e-12
    assert abs(ccsd.energy(S.f0, S.g, T1, T2) - Eb) < 1e-12


@pytest.mark.parametrize("o,v", CASES)
def test_lambda_residual(o, v):
    S, _, (T1, T2, L1, L2) = _setup(o, v, 2)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    L1b, L2b = bf.l_residual(T1, T2, L1, L2)
    R1, R2 = ccsd.l_residual(S.f0, S.g, T1, T2, L1, L2)
    assert np.max(np.abs(L1b)) > 1e-2
    assert np.max(np.abs(R1 - L1b)) < 1e-12
    assert np.max(np.abs(R2 - L2b)) < 1e-12


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3), (2, 4)])
def test_one_body_operator_residuals(o, v):
    """Residuals of a bare one-body operator (the dipole coupling alone; used by the kick)."""
    S, _, (T1, T2, L1, L2) = _setup(o, v, 3)
    m = S.mu[2]
    bf = bruteforce.BruteForce(m, None, 2 * o)
    R1b, R2b, _ = bf.t_residual(T1, T2)
    L1b, L2b = bf.l_residual(T1, T2, L1, L2)
    R1, R2 = ccsd.t_residual(m, None, T1, T2)
    Q1, Q2 = ccsd.l_residual(m, None, T1, T2, L1, L2)
    for a, b in ((R1, R1b), (R2, R2b), (Q1, L1b), (Q2, L2b)):
        assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3), (2, 4)])
def test_dipole_expectation(o, v):
    S, cs, (T1, T2, L1, L2) = _setup(o, v, 4)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * o)
    mu = ccsd.dipole(S, *cs)
    for a in range(3):
        ref = bf.expectation(S.mu[a], T1, T2, L1, L2)
        assert abs(mu[a] - ref) < 1e-12
    assert np.max(np.abs(mu.imag)) > 1e-6  # complex in general away from the ground state


def test_closed_shell_map_roundtrip():
    rng = np.random.default_rng(0)
    from synth import random_amplitudes
    x1, x2 = random_amplitudes(3, 4, rng)
    X1, X2 = spinorb.cs_to_so(x1, x2)
    # antisymmetry of the spin-orbital doubles
    assert np.allclose(X2, -X2.swapaxes(0, 1))
    assert np.allclose(X2, -X2.swapaxes(2, 3))
    y1, y2 = spinorb.so_to_cs(X1, X2, 3, 4)
    assert np.array_equal(y1, x1) and np.array_equal(y2, x2)


def test_spin_adapted_rhs_is_closed_shell():
    """The spin-orbital RHS of a closed-shell state stays in the closed-shell manifold."""
    o, v = 2, 3
    S, _, (T1, T2, L1, L2) = _setup(o, v, 5)
    R1, R2 = ccsd.t_residual(S.f0, S.g, T1, T2)
    r1, r2 = spinorb.so_to_cs(R1, R2, o, v)
    Q1, Q2 = spinorb.cs_to_so(r1, r2)
    assert np.max(np.abs(Q1 - R1)) < 1e-13 and np.max(np.abs(Q2 - R2)) < 1e-13
    P1, P2 = ccsd.l_residual(S.f0, S.g, T1, T2, L1, L2)
    p1, p2 = spinorb.so_to_cs(P1, P2, o, v)
    Q1, Q2 = spinorb.cs_to_so(p1, p2)
    assert np.max(np.abs(Q1 - P1)) < 1e-13 and np.max(np.abs(Q2 - P2)) < 1e-13
    # closed-shell pair symmetry of the doubles
    assert np.max(np.abs(r2 - r2.transpose(1, 0, 3, 2))) < 1e-13
