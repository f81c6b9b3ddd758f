"""Pins of the oracle's spatial -> spin-orbital integral map (no GPU).

``spinorb.so_one_body`` and ``spinorb.so_antisym_eri`` build the spin-orbital Fock matrix and
antisymmetrised integrals that both the factorised equations and the brute-force determinant
evaluator consume, so the brute-force pins cannot see a mistake in them. These tests compare the
determinant-space Hamiltonian built from them with quantities written straight from the spatial
chemists' integrals (pq|rs) and Fock matrix f, with no spin orbitals involved:

* the closed-shell reference energy  E_ref = 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)]  with the
  spatial core matrix  h = f - sum_k [2 (pq|kk) - (pk|kq)]  (the normal-ordered Fock operator of
  the Hamiltonian is f, the convention of the paper's field-dressed Fock matrix);
* the whole two-electron spectrum: for two electrons the Hamiltonian acts on spatial pair
  functions phi_p(1) phi_q(2) as  H_{pq,rs} = h_pr d_qs + d_pr h_qs + (pr|qs); its symmetric
  (singlet) and antisymmetric (triplet) parts must reproduce the determinant-space spectrum, each
  triplet level three times (M_S = -1, 0, 1). A transposed chemists'/physicists' index, a dropped
  exchange term or a wrong spin delta changes these eigenvalues.
"""
import numpy as np
import pytest

from oracle import bruteforce, ccsd
from synth import make_system, random_symmetric


def _system(o, v, seed):
    eri, fock, mu = make_system(o, v, seed=seed)
    fock = fock + random_symmetric(o + v, 0.1, np.random.default_rng(500 + seed))  # non-diagonal
    return eri, fock, mu


def _spatial_core(eri, fock, o):
    """h = f - sum_k [2 (pq|kk) - (pk|kq)] over the doubly occupied k."""
    J = np.einsum("pqkk->pq", eri[:, :, :o, :o])
    K = np.einsum("pkkq->pq", eri[:, :o, :o, :])
    return fock - (2.0 * J - K)


def _brute(eri, fock, o, v):
    S = ccsd.SpinOrbitalSystem(eri, fock, np.zeros((3, o + v, o + v)), o, v)
    return bruteforce.BruteForce(S.f0, S.g, 2 * o)


def _determinant_hamiltonian(eri, fock, o, v):
    bf = _brute(eri, fock, o, v)
    dim = bf.space.dim
    cols = [bruteforce._apply_hamiltonian(bf.space, bf.h, bf.g, np.eye(dim)[:, k].astype(complex))
            for k in range(dim)]
    return np.column_stack(cols), bf.space.ref


@pytest.mark.parametrize("o,v,seed", [(1, 3, 0), (2, 3, 1), (2, 4, 2), (3, 3, 3)])
def test_reference_energy_closed_shell_formula(o, v, seed):
    eri, fock, _ = _system(o, v, seed)
    bf = _brute(eri, fock, o, v)
    vac = bf.space.vac()
    e_det = (vac @ bruteforce._apply_hamiltonian(bf.space, bf.h, bf.g, vac)).real
    h = _spatial_core(eri, fock, o)
    e_ref = 2.0 * np.trace(h[:o, :o])
    for i in range(o):
        for j in range(o):
            e_ref += 2.0 * eri[i, i, j, j] - eri[i, j, j, i]
    assert abs(e_det - e_ref) < 1e-12
    # equivalently sum of occupied Fock energies minus the double-counted two-electron part
    e2 = 2.0 * np.trace(fock[:o, :o]) - sum(2.0 * eri[i, i, j, j] - eri[i, j, j, i]
                                            for i in range(o) for j in range(o))
    assert abs(e_det - e2) < 1e-12


@pytest.mark.parametrize("v,seed", [(3, 4), (4, 5), (5, 6)])
def test_two_electron_spectrum_from_spatial_pairs(v, seed):
    o = 1
    n = o + v
    eri, fock, _ = _system(o, v, seed)
    H, _ = _determinant_hamiltonian(eri, fock, o, v)
    assert np.allclose(H, H.conj().T, atol=1e-13)
    w_det = np.sort(np.linalg.eigvalsh(H))

    h = _spatial_core(eri, fock, o)
    I = np.eye(n)
    # H_{(p,q),(r,s)} = h_pr d_qs + d_pr h_qs + (pr|qs)
    Hpair = (np.einsum("pr,qs->pqrs", h, I) + np.einsum("pr,qs->pqrs", I, h)
             + eri.transpose(0, 2, 1, 3)).reshape(n * n, n * n)
    swap = np.zeros((n * n, n * n))
    for p in range(n):
        for q in range(n):
            swap[p * n + q, q * n + p] = 1.0
    Psym, Panti = 0.5 * (np.eye(n * n) + swap), 0.5 * (np.eye(n * n) - swap)

    def restricted(P):
        w, U = np.linalg.eigh(P)
        B = U[:, w > 0.5]  # orthonormal basis of the subspace
        return np.linalg.eigvalsh(B.T @ Hpair @ B)

    singlets, triplets = restricted(Psym), restricted(Panti)
    assert singlets.size == n * (n + 1) // 2 and triplets.size == n * (n - 1) // 2
    w_pair = np.sort(np.concatenate([singlets, triplets, triplets, triplets]))
    assert w_pair.size == w_det.size
    assert np.max(np.abs(w_pair - w_det)) < 1e-12


def test_spectrum_pin_detects_a_transposed_integral():
    """The spectrum comparison fails for the plausible mistake it is there to catch:
    using (pq|rs) as if it were <pq|rs>."""
    o, v = 1, 3
    n = o + v
    eri, fock, _ = _system(o, v, 7)
    wrong = eri.transpose(0, 2, 1, 3)  # (pq|rs) -> (pr|qs): the chemists'/physicists' swap applied twice
    H_bad, _ = _determinant_hamiltonian(wrong, fock, o, v)
    H_ok, _ = _determinant_hamiltonian(eri, fock, o, v)
    assert np.max(np.abs(np.linalg.eigvalsh(H_bad) - np.linalg.eigvalsh(H_ok))) > 1e-4
