"""Differentiable dipole trajectories: the library's adjoint behind ``torch.autograd.Function``.

``pulse_dipole_trajectory(R, params, y0, n, t0, dt, nsteps, every)`` propagates ``y0`` with RK4 under
the Gaussian pulse of Eq. field with parameters ``params = (E0, omega, sigma, t0_pulse)`` along ``n``
and returns the complex dipole (x, y, z) at the ``nsteps + 1`` grid times. Its backward is the
discrete adjoint of the RK4 map (``rtcc_step_rk4_vjp``) with the dipole cotangents injected at every
grid point (``rtcc_dipole_vjp``); the forward keeps only a state checkpoint every ``every`` steps and
the backward recomputes each segment's states from its checkpoint (one segment held at a time).
Gradients flow to ``params`` (float64) and to ``y0`` (complex128, the real-loss convention
dL/dRe + i dL/dIm). All arithmetic runs in the library; this module only orders the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Field


class _PulseTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, y0, R, n, t0, dt, nsteps, every):
        p = [float(x) for x in params.detach().cpu().tolist()]
        fld = Field.gaussian(p[0], p[1], p[2], p[3], n)
        y = y0.detach().clone()
        mu = torch.zeros((nsteps + 1, 6), dtype=torch.float64, device=y.device)
        cps = []
        s = 0
        while s < nsteps:
            k = min(every, nsteps - s)
            cps.append(y.clone())
            R.propagate_rk4(y, t0 + s * dt, dt, k, fld, mu[s:s + k + 1])
            s += k
        if nsteps == 0:
            R.dipole_dev(y, mu[0])
            cps.append(y.clone())
        ctx.R, ctx.fld, ctx.cps = R, fld, cps
        ctx.t0, ctx.dt, ctx.nsteps, ctx.every = t0, dt, nsteps, every
        ctx.pdev = params.device
        return torch.complex(mu[:, 0::2], mu[:, 1::2])

    @staticmethod
    def backward(ctx, gmu):
        R, fld, cps = ctx.R, ctx.fld, ctx.cps
        t0, dt, nsteps, every = ctx.t0, ctx.dt, ctx.nsteps, ctx.every
        g = gmu.detach().to("cpu").numpy()
        ybar = R.new_state()
        pbar = np.zeros(4)
        for seg in range(len(cps) - 1, -1, -1):
            s0 = seg * every
            k = min(every, nsteps - s0)
            states = [cps[seg]]
            for i in range(k):
                y = states[-1].clone()
                R.step_rk4(y, t0 + (s0 + i) * dt, dt, fld)
                states.append(y)
            for i in range(k, 0, -1):
                idx = s0 + i
                if np.any(g[idx]):
                    R.dipole_vjp(states[i], g[idx], ybar)
                R.step_rk4_vjp(states[i - 1], t0 + (idx - 1) * dt, dt, fld, ybar, pbar)
            del states
        if np.any(g[0]):
            R.dipole_vjp(cps[0], g[0], ybar)
        return (torch.as_tensor(pbar, dtype=torch.float64, device=ctx.pdev), ybar,
                None, None, None, None, None, None)


def pulse_dipole_trajectory(R, params, y0, n, t0, dt, nsteps, every=20):
    """Complex dipole (nsteps + 1, 3) of an RK4 propagation under a Gaussian pulse; differentiable."""
    return _PulseTrajectory.apply(params, y0, R, list(n), float(t0), float(dt), int(nsteps), int(every))


def integrated_dipole(mu, dt, component=2):
    """Trapezoid integral of Re mu_component over the uniform grid: the scalar loss of the gradient tests."""
    x = mu[:, component].real
    return dt * (x.sum() - 0.5 * (x[0] + x[-1]))
