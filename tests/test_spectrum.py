"""Pins of the absorption-spectrum readout (no GPU) on analytic damped sinusoids.

For d_k = sum_n A_n exp(-G_n t_k) sin(w_n t_k) on t_k = k dt, the windowed sum
sum_k d_k w_k exp(i w t_k) dt is a sum of geometric series, so the spectrum S(w) and the exact
position of each of its maxima are known in closed form (up to a 1-D maximisation); the FFT
pipeline, the padding, the window and the parabolic peak refinement must reproduce them.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from paper_2205_05175_amd import spectrum as sp

DT, T, KAPPA = 0.02, 100.0, 1e-3


def _signal(comps, n):
    t = DT * np.arange(n)
    return t, sum(A * np.exp(-G * t) * np.sin(w * t) for A, G, w in comps)


def _closed_form(comps, n, omega, gamma):
    """omega Im[sum_k d_k e^{-gamma t_k} e^{i omega t_k} dt] / kappa by geometric series."""
    total = 0j
    for A, G, w in comps:
        for sgn in (+1, -1):  # sin = (e^{iwt} - e^{-iwt}) / 2i
            r = np.exp((-(G + gamma) + 1j * (omega + sgn * w)) * DT)
            total = total + sgn * A / 2j * (1 - r ** n) / (1 - r) * DT
    return omega * total.imag / KAPPA


COMPS = [(1e-3, 0.0, 0.731), (4e-4, 0.01, 1.517), (2e-4, 0.0, 2.868), (6e-4, 0.02, 4.402)]


def test_fft_spectrum_equals_direct_sum():
    n = int(round(T / DT)) + 1
    _, d = _signal(COMPS, n)
    w, S = sp.absorption(d, DT, KAPPA)
    gamma = sp.WINDOW_DECAY / T
    idx = np.linspace(5, w.size - 5, 40).astype(int)
    ref = np.array([_closed_form(COMPS, n, w[j], gamma) for j in idx])
    assert np.max(np.abs(S[idx] - ref)) < 1e-9 * np.max(np.abs(S))
    assert w[-1] <= 10.0 and w[0] > 0


def test_peaks_match_closed_form_maxima():
    n = int(round(T / DT)) + 1
    _, d = _signal(COMPS, n)
    w, S = sp.absorption(d, DT, KAPPA)
    peaks = sp.find_peaks(w, S)
    gamma = sp.WINDOW_DECAY / T
    assert len(peaks) == len(COMPS)
    for p, (A, G, w0) in zip(sorted(peaks, key=lambda q: q.omega), COMPS):
        res = minimize_scalar(lambda x: -abs(_closed_form(COMPS, n, x, gamma)), bounds=(w0 - 0.05, w0 + 0.05),
                              method="bounded", options={"xatol": 1e-10})
        assert abs(p.omega - res.x) < 2e-5, (p.omega, res.x)
        assert abs(p.omega - w0) < 5e-3  # window and damping move a line only slightly


def test_nonzero_start_time_and_phase():
    """Samples starting at t0 != 0: the FFT carries the e^{i w t0} phase."""
    n = 2001
    t0 = 0.7
    t = t0 + DT * np.arange(n)
    d = 1e-3 * np.sin(1.3 * t)
    w, S = sp.absorption(d, DT, KAPPA, t0=t0)
    gamma = sp.WINDOW_DECAY / ((n - 1) * DT)
    j = np.argmin(np.abs(w - 1.0))
    direct = w[j] * np.sum(d * np.exp(-gamma * (t - t0)) * np.exp(1j * w[j] * t) * DT).imag / KAPPA
    assert abs(S[j] - direct) < 1e-9 * abs(direct)


def test_matching_reports_shift_and_unmatched():
    n = int(round(T / DT)) + 1
    _, d = _signal(COMPS, n)
    shifted = [(A, G, w + 5e-5) for A, G, w in COMPS]
    _, d2 = _signal(shifted, n)
    cmp, pr, po = sp.compare_trajectories(d, d2, DT, KAPPA)
    assert cmp.ok and len(cmp.pairs) == len(COMPS)
    assert abs(cmp.max_shift - 5e-5) < 1e-5
    extra = COMPS + [(5e-4, 0.0, 6.3)]
    _, d3 = _signal(extra, n)
    cmp3, _, _ = sp.compare_trajectories(d, d3, DT, KAPPA)
    assert not cmp3.ok and len(cmp3.unmatched_other) == 1 and abs(cmp3.unmatched_other[0] - 6.3) < 5e-3
    # identical trajectories: zero shift
    cmp0, _, _ = sp.compare_trajectories(d, d.copy(), DT, KAPPA)
    assert cmp0.ok and cmp0.max_shift == 0.0


def test_spline_resampling_of_adaptive_samples():
    rng = np.random.default_rng(0)
    steps = rng.uniform(0.05, 0.15, size=800)
    t = np.concatenate([[0.0], np.cumsum(steps)])
    t = t[t <= 60.0]
    f = lambda x: 1e-3 * np.sin(0.9 * x) + 5e-4 * np.cos(2.1 * x + 0.3)
    grid, x = sp.resample_uniform(t, f(t), DT, t_end=t[-1])
    assert abs(grid[1] - grid[0] - DT) < 1e-15 and grid[-1] <= t[-1] + 1e-12
    # not-a-knot cubic: error ~ h^4 f'''' / 384 with h <= 0.15 and |f''''| <= 1e-2
    assert np.max(np.abs(x - f(grid))) < 1e-7
    with pytest.raises(ValueError):
        sp.resample_uniform([0.0, 0.1, 0.1], [0, 1, 2], DT)


def test_noise_samples_are_bounded_and_seeded():
    a = sp.uniform_noise(10000, 3e-5, 7)
    assert np.abs(a).max() <= 3e-5 and np.abs(a).max() > 2.9e-5
    assert np.array_equal(a, sp.uniform_noise(10000, 3e-5, 7))
    assert abs(a.mean()) < 3e-5 * 0.05  # centred


def test_noise_change_is_linear_and_bounded():
    """The FFT is linear: the spectrum change is m times the spectrum of the unit noise pattern, and
    |dS(w)| <= w m sum_k exp(-gamma t_k) dt / kappa (every sample moves by at most m)."""
    n = int(round(T / DT)) + 1
    _, d = _signal(COMPS, n)
    w, s0 = sp.absorption(d, DT, KAPPA)
    unit = sp.uniform_noise(n, 1.0, 3)
    ds = {}
    for m in (1e-7, 1e-5):
        _, s1 = sp.absorption(d + m * unit, DT, KAPPA)
        ds[m] = s1 - s0
    assert np.allclose(ds[1e-5], 100.0 * ds[1e-7], rtol=1e-6, atol=1e-9 * np.abs(ds[1e-5]).max())
    gamma = sp.WINDOW_DECAY / T
    wsum = np.sum(np.exp(-gamma * DT * np.arange(n))) * DT
    assert np.all(np.abs(ds[1e-5]) <= w * 1e-5 * wsum / KAPPA * (1 + 1e-12))


def test_noise_study_threshold():
    """Noise far below the signal leaves every peak in place; noise of the signal's size does not."""
    n = int(round(T / DT)) + 1
    _, d = _signal(COMPS, n)
    res = sp.noise_study(d, DT, KAPPA, [1e-10, 1e-8, 1e-3], seed=1)
    assert res[0].unchanged and res[0].comparison.max_shift < 1e-6 and res[0].max_rel_change < 1e-5
    assert res[1].unchanged and res[1].max_rel_change < 1e-3
    assert not res[2].unchanged and res[2].max_rel_change > 0.1
    assert res[0].max_rel_change < res[1].max_rel_change < res[2].max_rel_change
