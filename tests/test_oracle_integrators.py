"""Pins of the oracle's Runge-Kutta integrators and field shapes (no GPU)."""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import field, integrators as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_tableau_row_sums():
    """Explicit tableaux: every row of A sums to its c (the corrected Cash-Karp tableau included)."""
    assert all(x == 0 for x in I.butcher_row_sums([Fr(0), Fr(1, 2), Fr(1, 2), Fr(1)],
                                                  [[], [Fr(1, 2)], [Fr(0), Fr(1, 2)], [Fr(0), Fr(0), Fr(1)]]))
    assert all(x == 0 for x in I.butcher_row_sums(I.CK_C, I.CK_A))


def test_printed_cash_karp_tableau_is_inconsistent():
    """The tableau as printed in Eq. ck-k (c4=1, c5=3/5, a42=+9/10, a63=-575/13824) fails the row sums."""
    c = list(I.CK_C)
    A = [list(r) for r in I.CK_A]
    c[3], c[4] = Fr(1), Fr(3, 5)
    A[3][1] = Fr(9, 10)
    A[5][2] = Fr(-575, 13824)
    bad = [x for x in I.butcher_row_sums(c, A) if x != 0]
    assert len(bad) >= 3


def _order_conditions(b, c, A):
    """Classical order conditions up to order 5 (the 17 rooted trees), returned as residuals."""
    s = len(b)
    b = [Fr(x) for x in b]
    c = [Fr(x) for x in c]
    A = [[Fr(A[i][j]) if j < len(A[i]) else Fr(0) for j in range(s)] for i in range(s)]

    def Av(x):
        return [sum(A[i][j] * x[j] for j in range(s)) for i in range(s)]

    def dot(x, y):
        return sum(p * q for p, q in zip(x, y))

    def mul(*xs):
        out = [Fr(1)] * s
        for x in xs:
            out = [p * q for p, q in zip(out, x)]
        return out

    one = [Fr(1)] * s
    c2, c3, c4 = mul(c, c), mul(c, c, c), mul(c, c, c, c)
    Ac, Ac2, Ac3 = Av(c), Av(c2), Av(c3)
    AAc, AAc2 = Av(Ac), Av(Ac2)
    AAAc = Av(AAc)
    conds = {
        1: [(dot(b, one), Fr(1))],
        2: [(dot(b, c), Fr(1, 2))],
        3: [(dot(b, c2), Fr(1, 3)), (dot(b, Ac), Fr(1, 6))],
        4: [(dot(b, c3), Fr(1, 4)), (dot(b, mul(c, Ac)), Fr(1, 8)), (dot(b, Ac2), Fr(1, 12)),
            (dot(b, AAc), Fr(1, 24))],
        5: [(dot(b, c4), Fr(1, 5)), (dot(b, mul(c2, Ac)), Fr(1, 10)), (dot(b, mul(c, Ac2)), Fr(1, 15)),
            (dot(b, mul(c, AAc)), Fr(1, 30)), (dot(b, mul(Ac, Ac)), Fr(1, 20)), (dot(b, Ac3), Fr(1, 20)),
            (dot(b, Av(mul(c, Ac))), Fr(1, 40)), (dot(b, AAc2), Fr(1, 60)), (dot(b, AAAc), Fr(1, 120))],
    }
    return {k: [x - y for x, y in v] for k, v in conds.items()}


def test_rk4_order_conditions():
    res = _order_conditions(I.RK4_B, I.RK4_C, I.RK4_A)
    for k in (1, 2, 3, 4):
        assert all(abs(float(x)) < 1e-15 for x in res[k])
    assert any(abs(float(x)) > 1e-3 for x in res[5])


def test_cash_karp_orders():
    """The 37/378 weights are fifth order, the 2825/27648 weights fourth order (the text swaps the labels)."""
    r5 = _order_conditions(I.CK_B5, I.CK_C, I.CK_A)
    r4 = _order_conditions(I.CK_B4, I.CK_C, I.CK_A)
    assert all(x == 0 for k in (1, 2, 3, 4, 5) for x in r5[k])
    assert all(x == 0 for k in (1, 2, 3, 4) for x in r4[k])
    assert any(x != 0 for x in r4[5])


def test_rk4_one_step_amplification():
    """One RK4 step on y' = lam y multiplies by the degree-4 Taylor polynomial of exp(h lam)."""
    lam = -0.3 + 2.1j
    for h in (0.05, 0.2, 0.7):
        y1 = I.rk4_step(lambda t, y: lam * y, 0.0, np.array([1.0 + 0j]), h)[0]
        z = h * lam
        assert abs(y1 - sum(z ** k / math.factorial(k) for k in range(5))) < 1e-14


def test_cash_karp_one_step_taylor():
    """The fifth-order CK solution matches exp(z) through z^5; the embedded one through z^4."""
    lam = 0.4 - 1.3j
    for h in (0.01, 0.02):
        y5, y4, _ = I.cashkarp_trial(lambda t, y: lam * y, 0.0, np.array([1.0 + 0j]), h)
        z = h * lam
        t5 = sum(z ** k / math.factorial(k) for k in range(6))
        t4 = sum(z ** k / math.factorial(k) for k in range(5))
        assert abs(y5[0] - t5) < 5 * abs(z) ** 6
        assert abs(y4[0] - t4) < 5 * abs(z) ** 5


def _integrate(step, f, y0, T, n):
    y, h = y0.copy(), T / n
    for k in range(n):
        y = step(f, k * h, y, h)
    return y


@pytest.mark.parametrize("which,order", [("rk4", 4), ("ck5", 5)])
def test_global_order_nonlinear(which, order):
    """Global error ratio on y' = y cos t (solution exp(sin t)) when halving h."""
    f = lambda t, y: y * np.cos(t)
    exact = math.exp(math.sin(2.0))
    if which == "rk4":
        step = I.rk4_step
    else:
        step = lambda f, t, y, h: I.cashkarp_trial(f, t, y, h)[0]
    errs = [abs(_integrate(step, f, np.array([1.0]), 2.0, n)[0] - exact) for n in (10, 20, 40)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert abs(math.log2(r2) - order) < 0.35 and abs(math.log2(r1) - order) < 0.5


def test_rk4_imaginary_axis_stability_bound():
    """|R4(i x)| <= 1 exactly up to x = 2 sqrt(2)."""
    R = lambda z: sum(z ** k / math.factorial(k) for k in range(5))
    assert abs(R(1j * 2 * math.sqrt(2) * (1 - 1e-9))) <= 1.0
    assert abs(R(1j * 2 * math.sqrt(2) * 1.01)) > 1.0


def test_cash_karp_controller():
    """Accept iff Delta <= eps; growth 0.84 (eps/Delta)^(1/5), shrink 0.84 (eps/Delta)^(1/4)."""
    assert I.ck_factor(1e-6, 1e-8) == pytest.approx(0.84 * 100 ** 0.2)
    assert I.ck_factor(1e-6, 1e-4) == pytest.approx(0.84 * 0.01 ** 0.25)
    assert I.ck_factor(1e-6, 0.0) == I.FACTOR_MAX
    assert I.ck_factor(1e-6, 1e30) == I.FACTOR_MIN
    lam = -1.0 + 8.0j
    f = lambda t, y: lam * y
    y, t, h = np.array([1.0 + 0j]), 0.0, 0.5
    rejected_total = 0
    while t < 3.0 - 1e-12:
        y, t, hu, h, rej = I.cashkarp_step(f, t, y, h, 1e-7, t_end=3.0)
        rejected_total += rej
    assert rejected_total >= 1  # the first trial (h = 0.5, |h lam| ~ 4) is rejected
    assert abs(y[0] - np.exp(lam * 3.0)) < 1e-5


# One Cash-Karp trial on y' = lam y multiplies y by these polynomials of z = h lam (from the
# corrected tableau: the fifth-order solution adds z^6 / 800 to the degree-5 Taylor polynomial).
def _R5(z):
    return sum(z ** k / math.factorial(k) for k in range(6)) + z ** 6 / 800


def _R4(z):
    return (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + Fr(10517, 1228800) * z ** 5
            + Fr(1771, 1638400) * z ** 6)


def test_cash_karp_amplification_polynomials():
    """Exact rational amplification of one trial (Fraction arithmetic through the tableau)."""
    for z in (Fr(1, 3), Fr(-7, 5), Fr(2)):
        k = []
        for i in range(6):
            yi = 1 + sum(I.CK_A[i][j] * z * k[j] for j in range(len(I.CK_A[i])))
            k.append(yi)  # f(y) = lam y, so h k_i = z y_i
        y5 = 1 + z * sum(b * x for b, x in zip(I.CK_B5, k))
        y4 = 1 + z * sum(b * x for b, x in zip(I.CK_B4, k))
        assert y5 == _R5(z) and y4 == _R4(z)


def test_cash_karp_propagation_sequence_closed_form():
    """On y' = lam y every Delta = |R5(z) - R4(z)| |y| is known in closed form, so the whole
    accept / reject / step-size sequence of the propagation, clipped to land on t_end, is predicted
    exactly and must be reproduced."""
    lam = -0.05 + 6.0j
    eps, t_end, h0 = 1e-7, 4.0, 0.3
    R5 = lambda z: complex(sum(z ** k / math.factorial(k) for k in range(6)) + z ** 6 / 800)
    c4 = [1, 1, 1 / 2, 1 / 6, 1 / 24, 10517 / 1228800, 1771 / 1638400]
    R4 = lambda z: sum(c * z ** k for k, c in enumerate(c4))
    # predicted sequence
    pred, y, t, h, nrej = [], 1.0 + 0j, 0.0, h0, 0
    while t < t_end:
        hh = min(h, t_end - t)
        z = hh * lam
        d = abs(R5(z) - R4(z)) * abs(y)
        fac = min(max(0.84 * (eps / d) ** (0.2 if d <= eps else 0.25), 0.1), 5.0)
        if d <= eps:
            y, t = y * R5(z), t + hh
            pred.append((t, y))
        else:
            nrej += 1
        h = hh * fac
    got = []
    yf, tf, nacc, nrj, _ = I.cashkarp_propagate(lambda tt, yy: lam * yy, 0.0, np.array([1.0 + 0j]), h0, eps,
                                                 t_end, on_accept=lambda tt, yy: got.append((tt, yy[0])))
    assert nacc == len(pred) and nrj == nrej and nrej >= 1
    assert tf == t_end
    # Delta is a difference of two O(1) numbers: its rounding (~1e-16 / 1e-7 relative) moves each h
    # by ~1e-10 relative, so the times and values agree to that level, the decisions exactly
    for (ta, ya), (tb, yb) in zip(got, pred):
        assert abs(ta - tb) < 1e-9 and abs(ya - yb) < 1e-8
    assert abs(yf[0] - np.exp(lam * t_end)) < 1e-5


def test_field_envelope_matches_paper_values():
    g = json.load(open(os.path.join(GOLDEN, "field_envelope.json")))
    for p in g["points"]:
        m = field.gaussian_envelope_magnitude(p["t"], g["E0"], g["sigma"], g["t0"])
        if "magnitude" in p:
            assert abs(m - p["magnitude"]) <= p["rel_tol"] * p["magnitude"]
        else:
            assert 0.1 * p["order_of_magnitude"] < m < 10 * p["order_of_magnitude"]


def test_gaussian_field_shape():
    n = np.array([0.0, 0.0, 1.0])
    E = field.gaussian(15.0, 0.01, 0.5, 5.0, 15.0, n)
    assert np.allclose(E, [0, 0, -0.01])  # peak value -E0 at the centre, cos = 1
    iso = np.ones(3) / math.sqrt(3)
    E = field.gaussian(12.0, 0.01, 0.5, 5.0, 15.0, iso)
    assert np.allclose(E, -0.01 * math.exp(-0.5 * 9 / 25) * math.cos(-1.5) * iso)


# ---- Fehlberg 4(5), the generic embedded driver, Gauss-Legendre ---------------------------------

def test_rkf45_orders():
    """Fehlberg's pair: consistent rows; the advancing weights are exactly fourth order (and not
    fifth), the embedded weights exactly fifth order."""
    assert all(x == 0 for x in I.butcher_row_sums(I.RKF45_C, I.RKF45_A))
    r4 = _order_conditions(I.RKF45_B4, I.RKF45_C, I.RKF45_A)
    r5 = _order_conditions(I.RKF45_B5, I.RKF45_C, I.RKF45_A)
    assert all(x == 0 for k in (1, 2, 3, 4) for x in r4[k])
    assert any(x != 0 for x in r4[5])
    assert all(x == 0 for k in (1, 2, 3, 4, 5) for x in r5[k])


def test_controller_factor_matches_paper_exponents():
    for d in (1e-9, 1e-7, 1e-6, 3e-6, 1e-3, 0.0, 1e30):
        assert I.controller_factor(1e-6, d, 4) == I.ck_factor(1e-6, d)
    assert I.controller_factor(1e-6, 1e-8, 2) == pytest.approx(0.84 * 100 ** (1 / 3))


@pytest.mark.parametrize("which,order", [("rkf4", 4), ("rkf5", 5)])
def test_rkf45_global_order(which, order):
    f = lambda t, y: y * np.cos(t)
    exact = math.exp(math.sin(2.0))
    b = I.RKF45_B4 if which == "rkf4" else I.RKF45_B5
    step = lambda f, t, y, h: I.rk_combine(y, h, b, I.rk_stages(f, t, y, h, I.RKF45_C, I.RKF45_A))
    # the fourth-order solution's leading error constant is small: asymptotic only from h = 0.1
    errs = [abs(_integrate(step, f, np.array([1.0]), 2.0, n)[0] - exact) for n in (20, 40, 80)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert abs(math.log2(r2) - order) < 0.35 and abs(math.log2(r1) - order) < 0.5


def test_embedded_driver_with_cash_karp_is_the_cash_karp_driver():
    f = lambda t, y: np.array([y[1], -np.sin(y[0]) + 0.3 * np.cos(1.7 * t)], dtype=complex)
    y0 = np.array([1.0 + 0j, 0.0 + 0j])
    a, b = [], []
    ra = I.cashkarp_propagate(f, 0.0, y0, 0.4, 1e-8, 6.0, on_accept=lambda t, y: a.append((t, y.copy())))
    rb = I.embedded_propagate(f, 0.0, y0, 0.4, 1e-8, 6.0, I.CK_C, I.CK_A, I.CK_B5, I.CK_B4, 4,
                              on_accept=lambda t, y: b.append((t, y.copy())))
    assert ra[2:] == rb[2:] and len(a) == len(b)
    assert all(ta == tb and np.array_equal(ya, yb) for (ta, ya), (tb, yb) in zip(a, b))


def test_rkf45_adaptive_propagation_accuracy():
    """The fourth-order advancing solution under the controller: y' = lam y to t = 4 with eps = 1e-8
    stays within a few eps per accepted step of the exact solution, and a larger first step is rejected."""
    lam = -0.05 + 6.0j
    y, t, nacc, nrej, _ = I.embedded_propagate(lambda t, y: lam * y, 0.0, np.array([1.0 + 0j]), 0.5, 1e-8, 4.0,
                                               I.RKF45_C, I.RKF45_A, I.RKF45_B4, I.RKF45_B5, 4)
    assert t == 4.0 and nrej >= 1
    assert abs(y[0] - np.exp(lam * 4.0)) < 10 * nacc * 1e-8


SQ3, SQ15 = math.sqrt(3.0), math.sqrt(15.0)
GL_CLOSED = {
    2: ([0.5 - SQ3 / 6, 0.5 + SQ3 / 6], [[0.25, 0.25 - SQ3 / 6], [0.25 + SQ3 / 6, 0.25]], [0.5, 0.5]),
    3: ([0.5 - SQ15 / 10, 0.5, 0.5 + SQ15 / 10],
        [[5 / 36, 2 / 9 - SQ15 / 15, 5 / 36 - SQ15 / 30], [5 / 36 + SQ15 / 24, 2 / 9, 5 / 36 - SQ15 / 24],
         [5 / 36 + SQ15 / 30, 2 / 9 + SQ15 / 15, 5 / 36]], [5 / 18, 4 / 9, 5 / 18]),
}


@pytest.mark.parametrize("s", [2, 3])
def test_gauss_legendre_closed_form(s):
    """The collocation construction gives the textbook two- and three-stage Gauss tableaux."""
    c, A, b = I.gauss_legendre_tableau(s)
    cc, AA, bb = GL_CLOSED[s]
    # (the construction integrates products of s - 1 linear factors: a few ulps of rounding)
    assert np.allclose(c, cc, atol=1e-15, rtol=0) and np.allclose(b, bb, atol=4e-15, rtol=0)
    assert np.allclose(A, AA, atol=4e-15, rtol=0)


@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_gauss_legendre_simplifying_assumptions(s):
    """B(2s) (quadrature exact to degree 2s-1) and C(s) (stage order s): together order 2s."""
    c, A, b = I.gauss_legendre_tableau(s)
    for k in range(1, 2 * s + 1):
        assert abs(np.dot(b, c ** (k - 1)) - 1.0 / k) < 1e-14
    for k in range(1, s + 1):
        assert np.allclose(A @ c ** (k - 1), c ** k / k, atol=1e-14, rtol=0)


def _pade(s, z):
    # diagonal Pade approximant of exp(z) of degree s (the stability function of s-stage Gauss)
    num = sum(math.factorial(2 * s - j) * math.factorial(s) / (math.factorial(2 * s) * math.factorial(j)
                                                               * math.factorial(s - j)) * z ** j for j in range(s + 1))
    return num / sum(math.factorial(2 * s - j) * math.factorial(s) / (math.factorial(2 * s) * math.factorial(j)
                                                                   * math.factorial(s - j)) * (-z) ** j
                     for j in range(s + 1))


@pytest.mark.parametrize("s", [2, 3])
def test_gauss_legendre_step_is_pade(s):
    """On y' = lam y the converged step multiplies y by the (s,s) Pade approximant of exp(h lam)."""
    c, A, b = I.gauss_legendre_tableau(s)
    lam = -0.4 + 3.0j
    for h in (0.02, 0.1):
        y1, it = I.implicit_rk_step(lambda t, y: lam * y, 0.0, np.array([1.0 + 0j]), h, c, A, b, 1e-15, 200)
        assert abs(y1[0] - _pade(s, h * lam)) < 1e-13 and it >= 2


@pytest.mark.parametrize("s", [2, 3])
def test_gauss_legendre_linear_system_and_unitarity(s):
    """y' = -i H y with a random Hermitian H: the fixed-point stages equal the direct solve of the
    linear stage equations, and 200 steps keep the norm (the Pade map of an imaginary-axis spectrum
    is unitary)."""
    rng = np.random.default_rng(5)
    n = 6
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = (M + M.conj().T) / 8
    J = -1j * H
    f = lambda t, y: J @ y
    c, A, b = I.gauss_legendre_tableau(s)
    y = rng.normal(size=n) + 1j * rng.normal(size=n)
    h = 0.05
    y1, _ = I.implicit_rk_step(f, 0.0, y, h, c, A, b, 1e-15, 200)
    big = np.eye(s * n, dtype=complex) - h * np.kron(A, J)
    K = np.linalg.solve(big, np.kron(np.ones(s), J @ y)).reshape(s, n)
    assert np.abs(y1 - (y + h * (b @ K))).max() < 1e-13
    nrm = np.linalg.norm(y)
    for _ in range(200):
        y, _ = I.implicit_rk_step(f, 0.0, y, h, c, A, b, 1e-15, 200)
    assert abs(np.linalg.norm(y) - nrm) < 1e-11 * nrm


@pytest.mark.parametrize("s,order", [(2, 4), (3, 6)])
def test_gauss_legendre_global_order(s, order):
    f = lambda t, y: y * np.cos(t)
    exact = math.exp(math.sin(2.0))
    c, A, b = I.gauss_legendre_tableau(s)
    step = lambda f, t, y, h: I.implicit_rk_step(f, t, y, h, c, A, b, 1e-16, 400)[0]
    ns = (4, 8, 16) if s == 3 else (8, 16, 32)
    errs = [abs(_integrate(step, f, np.array([1.0]), 2.0, n)[0] - exact) for n in ns]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert abs(math.log2(r2) - order) < 0.5 and abs(math.log2(r1) - order) < 0.6


def test_implicit_iteration_limit():
    c, A, b = I.gauss_legendre_tableau(2)
    with pytest.raises(RuntimeError):
        I.implicit_rk_step(lambda t, y: -40.0 * y, 0.0, np.array([1.0]), 0.2, c, A, b, 1e-12, 50)
