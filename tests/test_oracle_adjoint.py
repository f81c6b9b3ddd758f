"""Pins of the adjoint structure, on the oracle (CPU).

The GPU adjoint rests on three facts, each checked here against the spin-orbital oracle:

1. the right-hand side F is a polynomial of degree 4 in the state, so its Jacobian-vector product is
   the first Taylor coefficient of F(y + eps u), read exactly from four points on a circle;
2. F = S grad L (the equations of motion Eqs. derivT / derivL are the Lagrangian's gradient up to the
   swap S = [[0, -i G^-1], [i G^-1, 0]] with the closed-shell metric G), so the bilinear transpose of
   the Jacobian is J^T w = -S^-1 J (S w);
3. the dipole is the Lagrangian of the dipole operator (Eq. dipole), so grad mu_a = S^-1 F[mu_a, 0].

Plus the convergence of the stored finite-difference gradient of a pulse-driven trajectory.
"""
import json
import os

import numpy as np
import pytest

from oracle import ccsd
from synth import make_system, pack_state, random_state, random_symmetric, unpack_state

O, V = 2, 3
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system():
    eri, fock, mu = make_system(O, V, 1)
    fock = fock + random_symmetric(O + V, 0.05, np.random.default_rng(7))
    return ccsd.SpinOrbitalSystem(eri, fock, mu, O, V)


def _sym(y):
    t1, t2, l1, l2 = unpack_state(y, O, V)
    return pack_state(t1, 0.5 * (t2 + t2.transpose(1, 0, 3, 2)), l1, 0.5 * (l2 + l2.transpose(1, 0, 3, 2)))


def _rand(rng, n):
    return _sym(rng.normal(size=n) + 1j * rng.normal(size=n))


def _circle_coef1(f, y, u, m, r=0.3):
    w = np.exp(2j * np.pi * np.arange(m) / m)
    return sum(np.conj(w[j]) * f(y + r * w[j] * u) for j in range(m)) / (m * r)


def _metric(x, inverse):
    t1, t2, l1, l2 = unpack_state(x, O, V)
    g2 = (lambda a: (2 * a + a.transpose(0, 1, 3, 2)) / 3) if inverse else (lambda a: 2 * a - a.transpose(0, 1, 3, 2))
    f1 = 0.5 if inverse else 2.0
    return f1 * t1, g2(t2), f1 * l1, g2(l2)


def _S(x):
    t1, t2, l1, l2 = _metric(x, inverse=True)
    return pack_state(-1j * l1, -1j * l2, 1j * t1, 1j * t2)


def _Sinv(x):
    t1, t2, l1, l2 = _metric(x, inverse=False)
    return pack_state(-1j * l1, -1j * l2, 1j * t1, 1j * t2)


@pytest.fixture(scope="module")
def setup():
    S = _system()
    E = np.array([0.01, -0.02, 0.03])
    F = lambda y: pack_state(*ccsd.rhs(S, *unpack_state(y, O, V), E))
    y = pack_state(*random_state(O, V, 3))
    return S, E, F, y


def test_rhs_is_degree_four_polynomial(setup):
    S, E, F, y = setup
    rng = np.random.default_rng(5)
    u = _rand(rng, y.size)
    exact = _circle_coef1(F, y, u, 16)
    assert np.abs(_circle_coef1(F, y, u, 4) - exact).max() < 1e-13 * np.abs(exact).max()
    # three points alias the quartic coefficient: not exact
    assert np.abs(_circle_coef1(F, y, u, 3) - exact).max() > 1e-6 * np.abs(exact).max()
    # and the coefficient is the derivative: central difference agrees to its O(h^2)
    h = 1e-5
    fd = (F(y + h * u) - F(y - h * u)) / (2 * h)
    assert np.abs(fd - exact).max() < 1e-7 * np.abs(exact).max()


def test_hamiltonian_transpose_identity(setup):
    S, E, F, y = setup
    rng = np.random.default_rng(11)
    for _ in range(3):
        v, w = _rand(rng, y.size), _rand(rng, y.size)
        lhs = np.sum(w * _circle_coef1(F, y, v, 4))
        JTw = -_Sinv(_circle_coef1(F, y, _S(w), 4))
        rhs = np.sum(JTw * v)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_identity_fails_without_metric(setup):
    """The closed-shell metric matters: the plain swap [[0, -i], [i, 0]] does not transpose J."""
    S, E, F, y = setup
    rng = np.random.default_rng(12)
    v, w = _rand(rng, y.size), _rand(rng, y.size)
    plain = lambda x: pack_state(*[(-1j if k < 2 else 1j) * p for k, p in
                                   enumerate([unpack_state(x, O, V)[i] for i in (2, 3, 0, 1)])])
    lhs = np.sum(w * _circle_coef1(F, y, v, 4))
    rhs = np.sum(-plain(_circle_coef1(F, y, plain(w), 4)) * v)
    assert abs(lhs - rhs) > 1e-3 * abs(lhs)


def test_dipole_gradient_is_swapped_one_body_rhs(setup):
    S, E, F, y = setup
    rng = np.random.default_rng(13)
    for a in range(3):
        n = np.zeros(3)
        n[a] = 1.0
        Fm = pack_state(*ccsd.one_body_rhs(S, *unpack_state(y, O, V), n))
        grad = _Sinv(Fm)
        mu_a = lambda yy: np.array([ccsd.dipole(S, *unpack_state(yy, O, V))[a]])
        for _ in range(2):
            u = _rand(rng, y.size)
            d = _circle_coef1(mu_a, y, u, 8)[0]
            assert abs(np.sum(grad * u) - d) < 1e-12 * max(1.0, abs(d))


def test_stored_fd_gradient_converged():
    g = json.load(open(os.path.join(GOLDEN, "pulse_gradient_o2v6.json")))
    a, b = np.array(g["grad"]["1e-05"]), np.array(g["grad"]["2e-05"])
    assert np.abs(a - b).max() < 1e-8 * np.abs(a).max()
    # d L / d E0 at this small amplitude is dominated by linear response: L(E0) - L(0) ~ E0 dL/dE0
    assert g["grad"]["1e-05"][0] != 0.0
