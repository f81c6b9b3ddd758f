"""Linear absorption spectrum from a delta-kicked dipole trajectory (host-side analysis).

After a Dirac-delta kick E(t) = kappa delta(t) n (paper, Theory: "Linear absorption spectra from
RT-CC"), the induced dipole mu(t) - mu_gs is the linear response to the kick, its Fourier
transform divided by kappa is the polarisability alpha(omega), and the absorption cross section
is proportional to omega Im alpha(omega). This module turns the dipole samples the library
records into that curve and its peak positions, so that trajectories of different contraction
precisions or integrators can be compared peak by peak. It runs once per trajectory on the host
(NumPy FFT of 2^17 points) and is not part of the propagation.

Pipeline (the paper gives no window, padding or peak picking; these are the choices made here):

1. d_k = Re mu(t_k) - Re mu_gs on a uniform grid; adaptive (Cash-Karp) samples are first put on
   the grid by a not-a-knot cubic spline (the paper interpolates onto an evenly spaced grid
   without naming the method);
2. window w_k = exp(-gamma (t_k - t_0)) with gamma = 4.6 / T (1% left at the end, T the span);
3. zero padding to 2^17 samples;
4. S(omega) = omega Im[ sum_k d_k w_k exp(i omega t_k) dt ] / kappa on the FFT grid
   omega_j = 2 pi j / (N dt), 0 < omega_j <= omega_max;
5. peaks: local maxima of |S| above 5% of the largest |S|, each refined by a parabola through
   the three samples around it;
6. two peak lists are matched by mutual nearest neighbours; a peak without a partner within
   `match_window` is unmatched (a failure of the comparison).

Noise injection (Results, "Single-precision RT-CC"): the paper corrupts a double-precision dipole
trajectory with random noise of several magnitudes and looks for the magnitude at which the
spectrum starts to change. `noise_study` adds seeded uniform noise in [-m, m] to every sample (the
paper does not state the distribution; "magnitude cutoff" is read as the bound of a uniform
variate) and compares the noisy spectrum with the clean one: largest peak shift, peaks that lose
or gain a partner, peaks below the lowest clean peak (the low-frequency artefacts the paper
describes) and the largest change of S relative to its maximum.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NPAD = 1 << 17
WINDOW_DECAY = 4.6  # gamma * T


def resample_uniform(t, x, dt, t_end=None, t_start=None):
    """Not-a-knot cubic spline of the samples (t, x) on the grid t_start, t_start + dt, ... <= t_end."""
    from scipy.interpolate import CubicSpline
    t = np.asarray(t, float)
    x = np.asarray(x, float)
    if np.any(np.diff(t) <= 0):
        raise ValueError("sample times must increase strictly")
    t0 = t[0] if t_start is None else t_start
    t1 = t[-1] if t_end is None else t_end
    n = int(np.floor((t1 - t0) / dt + 1e-9)) + 1
    grid = t0 + dt * np.arange(n)
    return grid, CubicSpline(t, x, bc_type="not-a-knot")(grid)


def absorption(d, dt, kappa, t0=0.0, npad=NPAD, omega_max=10.0, gamma=None):
    """omega and S(omega) = omega Im FT[d w](omega) / kappa for 0 < omega <= omega_max.

    d: induced dipole samples at t0 + k dt (k = 0 .. len(d) - 1)."""
    d = np.asarray(d, float)
    n = d.size
    if n < 2:
        raise ValueError("need at least two samples")
    if npad < n:
        raise ValueError("padding shorter than the signal")
    span = (n - 1) * dt
    g = WINDOW_DECAY / span if gamma is None else gamma
    x = np.zeros(npad)
    x[:n] = d * np.exp(-g * dt * np.arange(n))
    # sum_k x_k e^{i w_j (t0 + k dt)} dt with w_j = 2 pi j / (N dt):  dt e^{i w_j t0} N ifft(x)_j
    F = np.fft.ifft(x) * npad * dt
    omega = 2.0 * np.pi * np.arange(npad) / (npad * dt)
    F = F * np.exp(1j * omega * t0)
    sel = (omega > 0) & (omega <= omega_max)
    return omega[sel], omega[sel] * F[sel].imag / kappa


@dataclass
class Peak:
    omega: float
    height: float  # signed value of S at the refined position


def find_peaks(omega, S, rel=0.05):
    """Local maxima of |S| with |S| >= rel * max|S|, refined by a three-point parabola."""
    omega = np.asarray(omega, float)
    a = np.abs(np.asarray(S, float))
    if a.size < 3:
        return []
    thr = rel * a.max()
    dw = omega[1] - omega[0]
    idx = np.nonzero((a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:]) & (a[1:-1] >= thr))[0] + 1
    out = []
    for j in idx:
        y0, y1, y2 = a[j - 1], a[j], a[j + 1]
        den = y0 - 2.0 * y1 + y2
        dlt = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        dlt = min(max(dlt, -0.5), 0.5)
        out.append(Peak(omega[j] + dlt * dw, float(np.sign(S[j]) * (y1 - 0.25 * (y0 - y2) * dlt))))
    return out


@dataclass
class PeakComparison:
    max_shift: float                  # largest |omega_other - omega_ref| over matched pairs
    pairs: list = field(default_factory=list)        # (omega_ref, omega_other)
    unmatched_ref: list = field(default_factory=list)
    unmatched_other: list = field(default_factory=list)

    @property
    def ok(self):
        return not self.unmatched_ref and not self.unmatched_other


def match_peaks(ref, other, match_window=0.02):
    """Mutual nearest-neighbour matching of two peak lists (Peak or float positions)."""
    r = np.array([p.omega if isinstance(p, Peak) else p for p in ref], float)
    o = np.array([p.omega if isinstance(p, Peak) else p for p in other], float)
    pairs, used_o = [], set()
    for i, w in enumerate(r):
        if o.size == 0:
            break
        j = int(np.argmin(np.abs(o - w)))
        back = int(np.argmin(np.abs(r - o[j])))
        if back == i and abs(o[j] - w) <= match_window:
            pairs.append((float(w), float(o[j])))
            used_o.add(j)
    matched_r = {p[0] for p in pairs}
    return PeakComparison(
        max_shift=max((abs(a - b) for a, b in pairs), default=0.0),
        pairs=pairs,
        unmatched_ref=[float(w) for w in r if float(w) not in matched_r],
        unmatched_other=[float(o[j]) for j in range(o.size) if j not in used_o])


def compare_trajectories(d_ref, d_other, dt, kappa, t0=0.0, rel=0.05, omega_max=10.0):
    """Spectra of two induced-dipole trajectories on the same grid and their peak comparison."""
    w, s_ref = absorption(d_ref, dt, kappa, t0=t0, omega_max=omega_max)
    _, s_oth = absorption(d_other, dt, kappa, t0=t0, omega_max=omega_max)
    p_ref, p_oth = find_peaks(w, s_ref, rel), find_peaks(w, s_oth, rel)
    return match_peaks(p_ref, p_oth), p_ref, p_oth


@dataclass
class NoiseResult:
    magnitude: float
    comparison: PeakComparison
    max_rel_change: float      # max |S_noisy - S_clean| / max |S_clean| over 0 < omega <= omega_max
    low_freq_peaks: int        # noisy-spectrum peaks below the lowest clean peak (minus the match window)

    @property
    def unchanged(self):
        return self.comparison.ok and self.low_freq_peaks == 0


def uniform_noise(n, magnitude, seed):
    """n seeded samples uniform in [-magnitude, magnitude]."""
    return magnitude * np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def noise_study(d, dt, kappa, magnitudes, seed=0, t0=0.0, rel=0.05, omega_max=10.0, match_window=0.02):
    """Spectra of d + uniform noise of each magnitude (same noise pattern, scaled) against the clean one."""
    d = np.asarray(d, float)
    w, s0 = absorption(d, dt, kappa, t0=t0, omega_max=omega_max)
    p0 = find_peaks(w, s0, rel)
    lowest = min((p.omega for p in p0), default=np.inf)
    unit = uniform_noise(d.size, 1.0, seed)
    out = []
    for m in magnitudes:
        _, s1 = absorption(d + m * unit, dt, kappa, t0=t0, omega_max=omega_max)
        p1 = find_peaks(w, s1, rel)
        out.append(NoiseResult(float(m), match_peaks(p0, p1, match_window),
                               float(np.abs(s1 - s0).max() / np.abs(s0).max()),
                               sum(1 for p in p1 if p.omega < lowest - match_window)))
    return out
