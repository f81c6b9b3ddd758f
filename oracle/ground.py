"""Ground-state CCSD and Lambda-CCSD amplitudes: the initial condition y0 (oracle).

Oracle (test infrastructure). The paper takes y0 to be the solution of the
ground-state T and Lambda equations (Theory, "Propagation of the RT-CC
equations"); the threshold is not stated, max|R| <= 1e-12 is used.

Method: Jacobi updates x <- x + R / D with orbital-energy differences
D_ia = f_ii - f_aa and D_ijab = f_ii + f_jj - f_aa - f_bb (diagonal of the
spatial Fock matrix), accelerated by DIIS on the update vectors. T is solved
first at zero field, then Lambda at the converged T starting from lambda = t.
"""
from __future__ import annotations

import numpy as np

from . import ccsd


class _DIIS:
    def __init__(self, nmax=8):
        self.nmax, self.x, self.e = nmax, [], []

    def extrapolate(self, x, e):
        self.x.append(x.copy())
        self.e.append(e.copy())
        if len(self.x) > self.nmax:
            self.x.pop(0)
            self.e.pop(0)
        m = len(self.x)
        if m < 2:
            return x
        B = -np.ones((m + 1, m + 1), complex)
        B[m, m] = 0.0
        for i in range(m):
            for j in range(m):
                B[i, j] = np.vdot(self.e[i], self.e[j])
        rhs = np.zeros(m + 1, complex)
        rhs[m] = -1.0
        try:
            c = np.linalg.solve(B, rhs)
        except np.linalg.LinAlgError:
            return x
        return sum(c[i] * self.x[i] for i in range(m))


def denominators(fock, o):
    eps = np.diag(fock)
    eo, ev = eps[:o], eps[o:]
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return d1, d2


def solve(sys: ccsd.SpinOrbitalSystem, fock_spatial, tol=1e-12, maxiter=200):
    """Return (t1, t2, l1, l2, e_corr) at zero field, closed-shell variables."""
    o, v = sys.o, sys.v
    d1, d2 = denominators(fock_spatial, o)
    n1 = o * v
    t1 = np.zeros((o, v), complex)
    t2 = np.zeros((o, o, v, v), complex)
    l1 = np.zeros((o, v), complex)
    l2 = np.zeros((o, o, v, v), complex)
    E0 = np.zeros(3)

    def pack(a, b):
        return np.concatenate([a.ravel(), b.ravel()])

    def unpack(x):
        return x[:n1].reshape(o, v), x[n1:].reshape(o, o, v, v)

    diis = _DIIS()
    for it in range(maxiter):
        r1, r2, _, _ = ccsd.residuals(sys, t1, t2, l1, l2, E0)
        if max(np.max(np.abs(r1)), np.max(np.abs(r2))) <= tol:
            break
        x = pack(t1 + r1 / d1, t2 + r2 / d2)
        e = pack(r1 / d1, r2 / d2)
        t1, t2 = unpack(diis.extrapolate(x, e))
    else:
        raise RuntimeError("T equations did not converge")
    l1, l2 = t1.copy(), t2.copy()
    diis = _DIIS()
    for it in range(maxiter):
        _, _, r1, r2 = ccsd.residuals(sys, t1, t2, l1, l2, E0)
        if max(np.max(np.abs(r1)), np.max(np.abs(r2))) <= tol:
            break
        x = pack(l1 + r1 / d1, l2 + r2 / d2)
        e = pack(r1 / d1, r2 / d2)
        l1, l2 = unpack(diis.extrapolate(x, e))
    else:
        raise RuntimeError("Lambda equations did not converge")
    from .spinorb import cs_to_so
    T1, T2 = cs_to_so(t1, t2)
    e_corr = ccsd.energy(sys.f0, sys.g, T1, T2)
    return t1, t2, l1, l2, e_corr
