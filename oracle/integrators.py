"""Explicit Runge-Kutta integrators for the RT-CC initial-value problem (oracle).

Oracle (test infrastructure). Follows the paper's "Propagation of the RT-CC
equations" subsection and "Comparison of numerical integrators":

* generic explicit RK (Eqs. rk_y, rk_k; Table tab:butcher): stage
  k_i = f(t_n + c_i h, y_n + h sum_j a_ij k_j), step y_{n+1} = y_n + h sum_i b_i k_i;
* classical RK4 (Eq. rk4truncation; the printed formula leaves out the factor h,
  which is restored here: y_{n+1} = y_n + (h/6)(k1 + 2k2 + 2k3 + k4));
* Cash-Karp embedded pair (Eqs. ck-k, ck-y). Three printed coefficients
  contradict the row-sum condition sum_j a_ij = c_i and are replaced by the
  values of Cash and Karp's own tableau: c4 = 3/5, c5 = 1, a42 = -9/10 and
  a63 = +575/13824. The weight set beginning 37/378 is the fifth-order one
  (the text labels it fourth order); the step advances with it;
* step-size control (Eqs. ck-h, ck-h-final): accept when Delta <= eps, with
  h_new = 0.84 h (eps/Delta)^(1/5); otherwise reject and retry with
  h_new = 0.84 h (eps/Delta)^(1/4). The error Delta is the largest complex
  modulus of y5 - y4 over the state. The factor is clamped to [0.1, 5]
  (not stated in the paper);
* Fehlberg's embedded 4(5) pair (Comparison of numerical integrators: six
  evaluations give a fifth- and a fourth-order solution, and the step advances
  with the fourth-order one), driven by the same controller;
* implicit Runge-Kutta with a full Butcher matrix (Introduction and Table
  tab:butcher: implicit methods couple the stages of one step and need an
  iterative solution), here Gauss-Legendre collocation. The paper gives no
  iteration: the stage equations k_i = f(t_n + c_i h, y_n + h sum_j a_ij k_j)
  are solved by fixed-point (Jacobi) sweeps from k_i = f(t_n, y_n), every
  sweep evaluating all s stages from the previous sweep's k, until
  h max_i max|k_i(new) - k_i(old)| <= tol.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

RK4_C = [0.0, 0.5, 0.5, 1.0]
RK4_A = [[], [0.5], [0.0, 0.5], [0.0, 0.0, 1.0]]
RK4_B = [1 / 6, 1 / 3, 1 / 3, 1 / 6]

CK_C = [Fr(0), Fr(1, 5), Fr(3, 10), Fr(3, 5), Fr(1), Fr(7, 8)]
CK_A = [
    [],
    [Fr(1, 5)],
    [Fr(3, 40), Fr(9, 40)],
    [Fr(3, 10), Fr(-9, 10), Fr(6, 5)],
    [Fr(-11, 54), Fr(5, 2), Fr(-70, 27), Fr(35, 27)],
    [Fr(1631, 55296), Fr(175, 512), Fr(575, 13824), Fr(44275, 110592), Fr(253, 4096)],
]
CK_B5 = [Fr(37, 378), Fr(0), Fr(250, 621), Fr(125, 594), Fr(0), Fr(512, 1771)]
CK_B4 = [Fr(2825, 27648), Fr(0), Fr(18575, 48384), Fr(13525, 55296), Fr(277, 14336), Fr(1, 4)]

SAFETY = 0.84
FACTOR_MIN, FACTOR_MAX = 0.1, 5.0


def rk_stages(f, t, y, h, c, A):
    """All stage derivatives k_i of an explicit tableau (Eq. rk_k)."""
    ks = []
    for i in range(len(c)):
        yi = y.copy()
        for j, a in enumerate(A[i]):
            if a != 0:
                yi = yi + h * float(a) * ks[j]
        ks.append(f(t + float(c[i]) * h, yi))
    return ks


def rk_combine(y, h, b, ks):
    """y + h sum_i b_i k_i (Eq. rk_y)."""
    out = y.copy()
    for bi, k in zip(b, ks):
        if bi != 0:
            out = out + h * float(bi) * k
    return out


def rk4_step(f, t, y, h):
    """One classical RK4 step."""
    ks = rk_stages(f, t, y, h, RK4_C, RK4_A)
    return rk_combine(y, h, RK4_B, ks)


def cashkarp_trial(f, t, y, h):
    """One Cash-Karp trial: (fifth-order solution, fourth-order solution, Delta)."""
    ks = rk_stages(f, t, y, h, CK_C, CK_A)
    y5 = rk_combine(y, h, CK_B5, ks)
    y4 = rk_combine(y, h, CK_B4, ks)
    delta = float(np.max(np.abs(y5 - y4))) if y5.size else 0.0
    return y5, y4, delta


def ck_factor(eps, delta):
    """Step-size factor of Eq. ck-h-final (with the clamp)."""
    if delta == 0.0:
        return FACTOR_MAX
    p = 0.2 if delta <= eps else 0.25
    fac = SAFETY * (eps / delta) ** p
    return min(max(fac, FACTOR_MIN), FACTOR_MAX)


def cashkarp_step(f, t, y, h, eps, t_end=None, max_tries=50):
    """Adaptive step: retry with shrinking h until accepted.

    Returns (y_new, t_new, h_used, h_next, n_rejected).
    """
    rejected = 0
    for _ in range(max_tries):
        hh = h if t_end is None else min(h, t_end - t)
        y5, _, delta = cashkarp_trial(f, t, y, hh)
        fac = ck_factor(eps, delta)
        if delta <= eps:
            return y5, t + hh, hh, hh * fac, rejected
        rejected += 1
        h = hh * fac
    raise RuntimeError("Cash-Karp step not accepted")


def cashkarp_propagate(f, t0, y0, h0, eps, t_end, on_accept=None, max_trials=1000000):
    """Adaptive Cash-Karp propagation from t0 to t_end (Eqs. ck-h, ck-h-final).

    Each trial uses hh = min(h, t_end - t), so the last step lands on t_end. An accepted trial
    advances y with the fifth-order solution and calls on_accept(t, y); after every trial
    h = hh * factor. Returns (y, t, n_accepted, n_rejected, h_next).
    """
    y, t, h = y0.copy(), t0, h0
    nacc = nrej = 0
    for _ in range(max_trials):
        if t >= t_end:
            return y, t, nacc, nrej, h
        hh = min(h, t_end - t)
        y5, _, delta = cashkarp_trial(f, t, y, hh)
        if not np.isfinite(delta):
            raise FloatingPointError("non-finite Cash-Karp error estimate")
        fac = ck_factor(eps, delta)
        if delta <= eps:
            y, t = y5, t + hh
            nacc += 1
            if on_accept is not None:
                on_accept(t, y)
        else:
            nrej += 1
        h = hh * fac
    raise RuntimeError("Cash-Karp propagation: too many trials")


def mixed_step_plan(t0, t_end, h1, h2, on_interval):
    """(start time, step size) list of mixed step-size RK4 (Results, strong fields): steps of h1 inside
    on_interval = (lo, hi) (the pulse "on", |t - nu| <= 5 sigma) and h2 outside; each phase ends with
    a shorter step landing on its boundary."""
    lo, hi = on_interval if on_interval is not None else (t_end, t_end)
    lo, hi = min(max(t0, lo), t_end), min(max(t0, hi), t_end)
    plan = []
    for a, b, h in ((t0, lo, h2), (lo, hi, h1), (hi, t_end, h2)):
        if b <= a:
            continue
        n = int(np.floor((b - a) / h * (1 + 1e-12)))
        plan += [(a + k * h, h) for k in range(n)]
        rem = (b - a) - n * h
        if rem > 1e-9 * h:
            plan.append((a + n * h, rem))
    return plan


def rk4_propagate_plan(f, y0, plan, on_step=None):
    """RK4 steps along a (start time, step size) plan; on_step(k, t_end_of_step, y) after each."""
    y = y0.copy()
    for k, (t, h) in enumerate(plan):
        y = rk4_step(f, t, y, h)
        if on_step is not None:
            on_step(k, t + h, y)
    return y


# Fehlberg's 4(5) pair (Fehlberg 1969; the published coefficients).
RKF45_C = [Fr(0), Fr(1, 4), Fr(3, 8), Fr(12, 13), Fr(1), Fr(1, 2)]
RKF45_A = [
    [],
    [Fr(1, 4)],
    [Fr(3, 32), Fr(9, 32)],
    [Fr(1932, 2197), Fr(-7200, 2197), Fr(7296, 2197)],
    [Fr(439, 216), Fr(-8), Fr(3680, 513), Fr(-845, 4104)],
    [Fr(-8, 27), Fr(2), Fr(-3544, 2565), Fr(1859, 4104), Fr(-11, 40)],
]
RKF45_B4 = [Fr(25, 216), Fr(0), Fr(1408, 2565), Fr(2197, 4104), Fr(-1, 5), Fr(0)]
RKF45_B5 = [Fr(16, 135), Fr(0), Fr(6656, 12825), Fr(28561, 56430), Fr(-9, 50), Fr(2, 55)]


def controller_factor(eps, delta, p):
    """Step factor of Eq. ck-h-final for a pair whose lower order is p: 0.84 (eps/Delta)^(1/(p+1))
    after an accepted trial, 0.84 (eps/Delta)^(1/p) after a rejected one, clamped to [0.1, 5]
    (p = 4 gives the paper's exponents 1/5 and 1/4)."""
    if delta == 0.0:
        return FACTOR_MAX
    e = 1.0 / (p + 1) if delta <= eps else 1.0 / p
    return min(max(SAFETY * (eps / delta) ** e, FACTOR_MIN), FACTOR_MAX)


def embedded_trial(f, t, y, h, c, A, b_adv, b_emb):
    """One trial of an embedded explicit pair: (advancing solution, Delta = max|y_adv - y_emb|)."""
    ks = rk_stages(f, t, y, h, c, A)
    y_adv = rk_combine(y, h, b_adv, ks)
    y_emb = rk_combine(y, h, b_emb, ks)
    delta = float(np.max(np.abs(y_adv - y_emb))) if y_adv.size else 0.0
    return y_adv, delta


def embedded_propagate(f, t0, y0, h0, eps, t_end, c, A, b_adv, b_emb, p, on_accept=None, max_trials=1000000):
    """Adaptive propagation with an embedded pair and the controller of Eq. ck-h-final; trial sizes
    are clipped to land on t_end as in cashkarp_propagate. Returns (y, t, n_accepted, n_rejected,
    h_next)."""
    y, t, h = y0.copy(), t0, h0
    nacc = nrej = 0
    for _ in range(max_trials):
        if t >= t_end:
            return y, t, nacc, nrej, h
        hh = min(h, t_end - t)
        y_adv, delta = embedded_trial(f, t, y, hh, c, A, b_adv, b_emb)
        if not np.isfinite(delta):
            raise FloatingPointError("non-finite error estimate")
        fac = controller_factor(eps, delta, p)
        if delta <= eps:
            y, t = y_adv, t + hh
            nacc += 1
            if on_accept is not None:
                on_accept(t, y)
        else:
            nrej += 1
        h = hh * fac
    raise RuntimeError("embedded propagation: too many trials")


def gauss_legendre_tableau(s):
    """s-stage Gauss-Legendre collocation: nodes c_i at the zeros of the shifted Legendre polynomial
    P_s(2c - 1), a_ij = integral over [0, c_i] and b_j = integral over [0, 1] of the j-th Lagrange
    basis polynomial on those nodes (order 2s). Returns (c, A, b) as float arrays."""
    x, w = np.polynomial.legendre.leggauss(s)
    c = (x + 1.0) / 2.0
    A = np.zeros((s, s))
    b = np.zeros(s)
    for j in range(s):
        lj = np.polynomial.Polynomial([1.0])
        for m in range(s):
            if m != j:
                lj = lj * np.polynomial.Polynomial([-c[m], 1.0]) / (c[j] - c[m])
        Lj = lj.integ()
        b[j] = Lj(1.0) - Lj(0.0)
        for i in range(s):
            A[i, j] = Lj(c[i]) - Lj(0.0)
    return c, A, b


def implicit_rk_step(f, t, y, h, c, A, b, tol, max_iter):
    """One step of an implicit Runge-Kutta method (full Butcher matrix A): the stage equations are
    solved by Jacobi fixed-point sweeps starting from k_i = f(t, y) until the largest change of
    h k_i in a sweep is <= tol. Returns (y_new, sweeps)."""
    s = len(c)
    k0 = f(t, y)
    ks = [k0] * s
    for it in range(1, max_iter + 1):
        new = []
        for i in range(s):
            yi = y.copy()
            for j in range(s):
                if A[i][j] != 0:
                    yi = yi + h * float(A[i][j]) * ks[j]
            new.append(f(t + float(c[i]) * h, yi))
        d = h * max(float(np.max(np.abs(new[i] - ks[i]))) if y.size else 0.0 for i in range(s))
        ks = new
        if d <= tol:
            return rk_combine(y, h, b, ks), it
    raise RuntimeError("implicit Runge-Kutta: stage iteration did not converge")


def butcher_row_sums(c, A):
    """sum_j a_ij - c_i for each row (zero for a consistent tableau)."""
    return [sum(A[i], Fr(0)) - c[i] for i in range(len(c))]
