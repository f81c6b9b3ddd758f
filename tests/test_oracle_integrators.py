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
