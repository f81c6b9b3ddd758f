"""External fields of the oracle: the Gaussian pulse and the Dirac-delta kick.

Oracle (test infrastructure).

* Gaussian envelope (Eq. field): E(t) = -E0 exp(-(t - t0)^2 / (2 sigma^2)) cos(omega (t - t0)) n,
  with the paper's centre nu written t0 here. n is a unit vector; the paper's
  isotropic choice (Eq. iso-field) is one value of it.
* Dirac-delta pulse (linear-absorption subsection): E(t) = kappa delta(t) n.
  Over a zero-width interval only the dipole term of H(t) = H0 - mu.E(t)
  acts, so the state just after the kick is the flow of
  dy/ds = kappa * F_mu(y) for s in [0, 1], where F_mu is the right-hand side
  of the operator n.mu alone (no two-electron part; module ``ccsd``) with the
  sign of the coupling absorbed. It is integrated with RK4 in 100 sub-steps.
"""
from __future__ import annotations

import numpy as np

from . import ccsd, integrators


def gaussian(t, E0, omega, sigma, t0, n):
    """Field vector E(t) of Eq. field."""
    env = np.exp(-0.5 * (t - t0) ** 2 / sigma ** 2)
    return -E0 * env * np.cos(omega * (t - t0)) * np.asarray(n, float)


def gaussian_envelope_magnitude(t, E0, sigma, t0):
    """|E0 * envelope| (the magnitudes the paper quotes while discussing Cash-Karp step sizes)."""
    return abs(E0) * np.exp(-0.5 * (t - t0) ** 2 / sigma ** 2)


def kick(sys, y_parts, kappa, n, substeps=100):
    """Apply a delta kick of strength kappa along unit vector n; returns the new (t1, t2, l1, l2).

    During the kick: dt/dt = -i R_T[f - E mu] contributes +i kappa R_T[n.mu, 0]
    per unit of the integrated field, and dlambda/dt contributes -i kappa R_L[n.mu, 0].
    ``ccsd.one_body_rhs`` returns (-i R_T[m], +i R_L[m]) for m = n.mu, so the kick
    derivative is -kappa times it.
    """
    o, v = sys.o, sys.v
    shapes = [(o, v), (o, o, v, v), (o, v), (o, o, v, v)]
    sizes = [int(np.prod(s)) for s in shapes]

    def pack(parts):
        return np.concatenate([np.ravel(p) for p in parts])

    def unpack(y):
        out, k = [], 0
        for s, m in zip(shapes, sizes):
            out.append(y[k:k + m].reshape(s))
            k += m
        return out

    def f(_s, y):
        d = ccsd.one_body_rhs(sys, *unpack(y), n)
        return -kappa * pack(d)

    y = pack(y_parts).astype(np.complex128)
    h = 1.0 / substeps
    for k in range(substeps):
        y = integrators.rk4_step(f, k * h, y, h)
    return unpack(y)
