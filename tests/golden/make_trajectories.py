"""Write the oracle's reference dipole trajectories used by the GPU trajectory tests.

Calls only the oracle (``oracle/``) and the seeded input generator (``synth``).

* delta_kick_o4v16.json  -- (o, v) = (4, 16), seed 0: ground state, delta kick of 1e-3 au
  along z, RK4 with dt = 0.05 au for 200 steps.
* gaussian_o5v19.json    -- (o, v) = (5, 19), seed 0: ground state, Gaussian pulse (Eq. field)
  E0 = 0.01 au, omega = 0.5 Eh, sigma = 5 au, centre t0 = 15 au, along z; RK4 with
  dt = 0.02 au for 1000 steps.

* cashkarp_o4v16        -- (o, v) = (4, 16), seed 0: ground state, delta kick of 1e-3 au along z,
  adaptive Cash-Karp from t = 0 to 3 au, h0 = 0.5 au (too long: the first trial is rejected), eps = 1e-6 (Eqs. ck-h, ck-h-final); the times
  and dipoles after every accepted step and the accepted / rejected counts.
* mixed_o2v4            -- (o, v) = (2, 4), seed 0: ground state in a strong Gaussian pulse
  (E0 = 100 au, omega = 0, sigma = 0.05 au, centre 0.25 au, along z), mixed step-size RK4 with
  h1 = 1e-3 au while |t - 0.25| <= 5 sigma and h2 = 0.01 au elsewhere, to t = 0.6 au; the ground
  state, and |T2| and the dipole after every step.

Each file stores the complex dipole (x, y, z) at every step end, reference part included,
plus the ground-state correlation energy. Usage: python tests/golden/make_trajectories.py [name]
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

CASES = {
    "delta_kick_o4v16": dict(o=4, v=16, seed=0, kick=1e-3, n=[0.0, 0.0, 1.0], dt=0.05, steps=200),
    "gaussian_o5v19": dict(o=5, v=19, seed=0, pulse=dict(E0=0.01, omega=0.5, sigma=5.0, t0=15.0),
                           n=[0.0, 0.0, 1.0], dt=0.02, steps=1000),
    "cashkarp_o4v16": dict(o=4, v=16, seed=0, kick=1e-3, n=[0.0, 0.0, 1.0], cashkarp=dict(h0=0.5, eps=1e-6,
                                                                                        t_end=3.0)),
    "mixed_o2v4": dict(o=2, v=4, seed=0, pulse=dict(E0=100.0, omega=0.0, sigma=0.05, t0=0.25),
                       n=[0.0, 0.0, 1.0], mixed=dict(h1=1e-3, h2=0.01, t_end=0.6)),
}


def _cplx(a):
    return [[z.real, z.imag] for z in np.ravel(a)]


def run(name):
    c = CASES[name]
    o, v = c["o"], c["v"]
    eri, fock, mu = make_system(o, v, c["seed"])
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    t1, t2, l1, l2, ecorr = ground.solve(S, fock)
    amps = (t1, t2, l1, l2)
    mu_gs = ccsd.dipole(S, *amps)
    if "kick" in c:
        amps = field.kick(S, amps, c["kick"], c["n"])
        Efun = lambda t: np.zeros(3)
    else:
        p = c["pulse"]
        Efun = lambda t: field.gaussian(t, p["E0"], p["omega"], p["sigma"], p["t0"], c["n"])
    f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, o, v), Efun(t)))
    y = pack_state(*amps)
    if "cashkarp" in c:
        ck = c["cashkarp"]
        ts, mus = [], []
        yf, tf, nacc, nrej, hn = integrators.cashkarp_propagate(
            f, 0.0, y, ck["h0"], ck["eps"], ck["t_end"],
            on_accept=lambda t, yy: (ts.append(t), mus.append(ccsd.dipole(S, *unpack_state(yy, o, v)))))
        out = dict(case=c, e_corr=float(ecorr.real), t=ts, mu=[_cplx(m) for m in mus], accepted=nacc,
                   rejected=nrej, h_next=hn, generator="tests/golden/make_trajectories.py (oracle, spin-orbital FP64)")
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh)
        print(f"{name}: {nacc} accepted, {nrej} rejected", flush=True)
        return
    if "mixed" in c:
        mx, p = c["mixed"], c["pulse"]
        plan = integrators.mixed_step_plan(0.0, mx["t_end"], mx["h1"], mx["h2"],
                                           (p["t0"] - 5 * p["sigma"], p["t0"] + 5 * p["sigma"]))
        norms = [float(np.linalg.norm(amps[1]))]
        mus = [ccsd.dipole(S, *amps)]

        def rec(k, t, yy):
            parts = unpack_state(yy, o, v)
            norms.append(float(np.linalg.norm(parts[1])))
            mus.append(ccsd.dipole(S, *parts))

        integrators.rk4_propagate_plan(f, y, plan, rec)
        out = dict(case=c, e_corr=float(ecorr.real), y0=_cplx(y), t=[0.0] + [t + h for t, h in plan],
                   t2norm=norms, mu=[_cplx(m) for m in mus],
                   generator="tests/golden/make_trajectories.py (oracle, spin-orbital FP64)")
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh)
        print(f"{name}: {len(plan)} steps, max |T2| {max(norms):.3f}", flush=True)
        return
    traj = [ccsd.dipole(S, *unpack_state(y, o, v))]
    t0 = time.time()
    for k in range(c["steps"]):
        y = integrators.rk4_step(f, k * c["dt"], y, c["dt"])
        traj.append(ccsd.dipole(S, *unpack_state(y, o, v)))
        if k % 50 == 0:
            print(f"{name}: step {k} ({time.time() - t0:.0f} s)", flush=True)
    traj = np.array(traj)
    out = dict(case=c, e_corr=float(ecorr.real), mu_ground=[[z.real, z.imag] for z in mu_gs],
               t=[k * c["dt"] for k in range(c["steps"] + 1)],
               mu=[[[z.real, z.imag] for z in row] for row in traj],
               generator="tests/golden/make_trajectories.py (oracle, spin-orbital FP64)")
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh)
    print(f"{name}: done", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        run(name)
