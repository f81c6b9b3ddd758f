"""Write the oracle's gradient of a pulse-driven, time-integrated dipole (used by the GPU adjoint tests).

Calls only the oracle (``oracle/``) and the seeded input generator (``synth``).

pulse_gradient_o2v6.json -- (o, v) = (2, 6), seed 0: ground state, then RK4 with dt = 0.05 au for
40 steps under the Gaussian pulse of Eq. field along z with (E0, omega, sigma, t0) = (0.05, 0.5, 0.5, 1.0).
Loss L = dt * trapezoid sum of Re mu_z over the 41 grid times. Stored: L and its gradient with respect
to (E0, omega, sigma, t0) by central differences of the oracle loss with h = 1e-5 and with h = 2e-5
(relative steps for omega, sigma and t0; absolute for E0), and the dipole trajectory.

Usage: python tests/golden/make_adjoint.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ccsd, field, ground, integrators  # noqa: E402
from synth import make_system, pack_state, unpack_state  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASE = dict(o=2, v=6, seed=0, params=[0.05, 0.5, 0.5, 1.0], n=[0.0, 0.0, 1.0], dt=0.05, steps=40)


def trajectory(S, y0, params, c):
    o, v = c["o"], c["v"]
    E0, om, sg, tc = params
    f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, o, v), field.gaussian(t, E0, om, sg, tc, c["n"])))
    y = y0
    mu = [ccsd.dipole(S, *unpack_state(y, o, v))]
    for k in range(c["steps"]):
        y = integrators.rk4_step(f, k * c["dt"], y, c["dt"])
        mu.append(ccsd.dipole(S, *unpack_state(y, o, v)))
    return np.array(mu)


def loss(mu, dt):
    x = mu[:, 2].real
    return dt * (x.sum() - 0.5 * (x[0] + x[-1]))


def main():
    c = CASE
    o, v = c["o"], c["v"]
    eri, fock, mu_ints = make_system(o, v, c["seed"])
    S = ccsd.SpinOrbitalSystem(eri, fock, mu_ints, o, v)
    t1, t2, l1, l2, ecorr = ground.solve(S, fock)
    y0 = pack_state(t1, t2, l1, l2)
    p0 = np.array(c["params"], float)
    t0 = time.time()
    mu = trajectory(S, y0, p0, c)
    L0 = loss(mu, c["dt"])
    grads = {}
    for h in (1e-5, 2e-5):
        g = np.zeros(4)
        for j in range(4):
            step = h if j == 0 else h * abs(p0[j])
            pp, pm = p0.copy(), p0.copy()
            pp[j] += step
            pm[j] -= step
            g[j] = (loss(trajectory(S, y0, pp, c), c["dt"]) - loss(trajectory(S, y0, pm, c), c["dt"])) / (2 * step)
        grads[str(h)] = g.tolist()
        print(f"h={h}: {g} ({time.time() - t0:.0f} s)", flush=True)
    out = dict(case=c, e_corr=float(ecorr.real), loss=float(L0), grad=grads,
               mu=[[[z.real, z.imag] for z in row] for row in mu],
               generator="tests/golden/make_adjoint.py (oracle, spin-orbital FP64, central differences)")
    with open(os.path.join(HERE, "pulse_gradient_o2v6.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
