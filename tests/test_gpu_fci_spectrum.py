"""Two-electron absorption spectrum on the GPU against full CI stick positions.

For two electrons CCSD is exact, so after a delta kick the RT-CCSD dipole is the TD-FCI dipole and its
absorption peaks sit at the dipole-allowed FCI excitation energies (the stick spectrum the paper
compares with, there from EOM-CCSD). System: synth (1,7), seed 0; kick 1e-3 au along z; RK4 at
dt = 0.05 au to t = 300 au in FP64, complex FP32 and split-BF16 (forced onto every product).

Checked:
* the FP64 GPU trajectory equals the exact TD-FCI dipole (eigen-decomposition of the determinant
  Hamiltonian of the oracle's brute-force module) to the RK4 error, and its spectrum peaks equal the
  exact signal's peaks through the same pipeline up to RK4's dispersion, w (h w)^4 / 120;
* every FCI excitation with oscillator weight omega |<n|mu_z|0>|^2 above 5% of the largest has a
  spectrum peak, and every peak above 5% has such an excitation, within a fifth of the window's
  Lorentzian half-width gamma = 4.6 / T = 0.015 Eh (an isolated peak lands ~1e-4 Eh from its
  excitation; a weak one beside a strong one is pulled by the strong one's tail, here by 1.1e-3 Eh);
* FP32 and split-BF16 spectra: the same peaks as FP64 within 1e-4 Eh.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from synth import make_system

pytestmark = pytest.mark.gpu

O, V, KAPPA, DT, T_END = 1, 7, 1e-3, 0.05, 300.0


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _fci():
    from oracle import bruteforce, ccsd
    eri, fock, mu = make_system(O, V, seed=0)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, O, V)
    bf = bruteforce.BruteForce(S.f0, S.g, 2 * O)
    dim = bf.space.dim
    cols = lambda A1, A2: np.column_stack(
        [bruteforce._apply_hamiltonian(bf.space, A1, A2, np.eye(dim)[:, k].astype(complex)) for k in range(dim)])
    H = cols(bf.h, bf.g)
    M = cols(S.mu[2], None)
    w, U = np.linalg.eigh(H)
    k0 = next(k for k in range(dim) if abs(U[bf.space.ref, k]) > 0.1)
    psi0 = U[:, k0]
    exc = w - w[k0]
    weight = exc * np.abs(U.conj().T @ M @ psi0) ** 2
    # exact kicked dynamics: psi(0+) = exp(i kappa mu_z) psi0, then exp(-i H t)
    c = U.conj().T @ (sla.expm(1j * KAPPA * M) @ psi0)
    MU = U.conj().T @ M @ U
    t = DT * np.arange(int(round(T_END / DT)) + 1)
    amps = np.exp(-1j * np.outer(t, w)) * c[None, :]
    mu_t = np.einsum("ti,ij,tj->t", amps.conj(), MU, amps).real
    mu_gs = float((psi0.conj() @ M @ psi0).real)
    return exc, weight, mu_t, mu_gs


def _gpu_trajectory(prec):
    import torch
    from paper_2205_05175_amd import RTCC, Field
    R = RTCC(*make_system(O, V, seed=0), O, V, prec)
    y = R.new_state()
    R.set_precision("fp64")
    R.ground_state(y, 1e-12, 200)
    mu_gs = R.dipole(y)[2].real
    R.kick(y, KAPPA, [0.0, 0.0, 1.0])
    R.set_precision(prec)
    n = int(round(T_END / DT))
    mu = torch.zeros((n + 1, 6), dtype=torch.float64, device="cuda")
    R.propagate_rk4(y, 0.0, DT, n, Field.none(), mu)
    torch.cuda.synchronize()
    out = mu[:, 4].cpu().numpy()
    R.close()
    return out, mu_gs


def test_two_electron_spectrum_matches_fci_sticks(monkeypatch):
    from paper_2205_05175_amd import spectrum as sp
    print("two-electron (1,7) spectrum vs FCI sticks, RK4 dt=0.05 to 300 au", flush=True)
    exc, weight, mu_exact, mu_gs_exact = _fci()
    d_exact = mu_exact - mu_gs_exact
    w, s_exact = sp.absorption(d_exact, DT, KAPPA)
    p_exact = sp.find_peaks(w, s_exact)

    mu64, gs64 = _gpu_trajectory("fp64")
    assert abs(gs64 - mu_gs_exact) < 1e-10
    err = np.abs(mu64 - mu_exact).max()
    print(f"  fp64 max |mu_z - TD-FCI| = {err:.2e} au", flush=True)
    assert err < 5e-5
    w, s64 = sp.absorption(mu64 - gs64, DT, KAPPA)
    p64 = sp.find_peaks(w, s64)
    cmp = sp.match_peaks(p_exact, p64)
    print(f"  peaks {[round(p.omega, 5) for p in p64]}; vs exact signal max shift {cmp.max_shift:.2e}", flush=True)
    # RK4 advances a mode of frequency w with phase error (h w)^5 / 120 per step, i.e. it oscillates at
    # w (1 - (h w)^4 / 120): allow twice that dispersion (3.7e-5 Eh at the 3.72 Eh peak) plus rounding
    assert cmp.ok
    for a, b in cmp.pairs:
        assert abs(a - b) <= 2 * a * (DT * a) ** 4 / 120 + 2e-6, (a, b)

    tol = 0.2 * 4.6 / T_END
    allowed = exc > 1e-6
    strong = allowed & (weight >= 0.05 * weight.max())
    for e in exc[strong]:
        assert min(abs(p.omega - e) for p in p64) < tol, f"FCI excitation {e:.5f} Eh has no peak"
    visible = exc[allowed & (weight >= 1e-3 * weight.max())]
    for p in p64:
        assert np.abs(visible - p.omega).min() < tol, f"peak {p.omega:.5f} Eh is no FCI excitation"

    # the same spectrum from complex-FP32 and split-BF16 contractions (split forced onto every product)
    monkeypatch.setenv("RTCC_BF16_MIN_FLOPS", "0")
    for prec in ("fp32", "bf16x3"):
        mu, gs = _gpu_trajectory(prec)
        _, s = sp.absorption(mu - gs, DT, KAPPA)
        c = sp.match_peaks(p64, sp.find_peaks(w, s))
        print(f"  {prec}: max |mu - fp64| = {np.abs(mu - mu64).max():.2e} au, peak shift {c.max_shift:.2e} Eh",
              flush=True)
        assert c.ok and c.max_shift < 1e-4
