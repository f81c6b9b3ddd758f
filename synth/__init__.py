"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
coupled-cluster arithmetic, so both the CPU oracle and the HIP path can take
their inputs from it without sharing any of the method.

Water-cluster-shaped Hamiltonian (closed shell, ``o`` doubly occupied and
``v`` virtual spatial orbitals, ``n = o + v``), drawn in this order from
``numpy.random.default_rng(seed)``:

1. occupied orbital energies ~ U[-1.5, -0.5] (sorted ascending),
2. virtual orbital energies ~ U[0.2, 3.0] (sorted ascending),
3. ``B`` ~ N(0, s^2) of shape ``(3n, n, n)``, made symmetric in its last
   two indices by mirroring the upper triangle, with s = 0.05 for n <= 24 and
   s = 0.05 * 24 / n beyond (see below),
4. dipole integrals ``mu`` ~ N(0, 0.3^2) of shape ``(3, n, n)``, mirrored the
   same way.

Then ``(pq|rs) = sum_Q B[Q,p,q] B[Q,r,s]`` (chemists' order, 8-fold symmetric)
and ``f = diag(eps_occ, eps_vir)`` with the occupied orbitals first.

Size scaling of ``s``: with a fixed s = 0.05 every exchange-type integral
(ia|ia) = sum_Q B[Q,i,a]^2 grows like 3n s^2 and the random off-diagonal ones like
sqrt(3n) s^2, so the correlation grows much faster than the system: at
(o, v) = (10, 38) the MP2 energy is -62 Eh and at (20, 76) -1739 Eh, and the CCSD
equations have no convergent solution. Scaling s by 24/n for n > 24 keeps the
coherent per-orbital sums (Fock-like dressings of size o^2 v (ia|jb)^2 / D)
independent of n, so the correlation energy grows linearly with the size, as
for a water cluster. Systems with n <= 24 are drawn exactly as before.
"""
from __future__ import annotations

import numpy as np


def _mirror_upper(x: np.ndarray) -> np.ndarray:
    """Copy the upper triangle (diagonal included) of the last two axes onto the lower one."""
    iu = np.triu(np.ones(x.shape[-2:], dtype=bool))
    return np.where(iu, x, np.swapaxes(x, -1, -2))


def b_sigma(n: int) -> float:
    """Standard deviation of the factors B for a system of n orbitals."""
    return 0.05 * min(1.0, 24.0 / n)


def make_system(o: int, v: int, seed: int = 0, dtype=np.float64):
    """Return ``(eri, fock, mu)``: eri ``(n,n,n,n)`` chemists' order, fock ``(n,n)``, mu ``(3,n,n)``."""
    n = o + v
    rng = np.random.default_rng(seed)
    eps_o = np.sort(rng.uniform(-1.5, -0.5, size=o))
    eps_v = np.sort(rng.uniform(0.2, 3.0, size=v))
    B = _mirror_upper(rng.normal(0.0, b_sigma(n), size=(3 * n, n, n)))
    mu = _mirror_upper(rng.normal(0.0, 0.3, size=(3, n, n)))
    Bm = B.reshape(3 * n, n * n)
    eri = (Bm.T @ Bm).reshape(n, n, n, n).astype(dtype)
    fock = np.diag(np.concatenate([eps_o, eps_v])).astype(dtype)
    return eri, fock, mu.astype(dtype)


def random_symmetric(n: int, scale: float, rng: np.random.Generator) -> np.ndarray:
    """A dense real symmetric ``n x n`` matrix with N(0, scale^2) entries."""
    return _mirror_upper(rng.normal(0.0, scale, size=(n, n)))


def random_amplitudes(o: int, v: int, rng: np.random.Generator, scale1: float = 0.05,
                      scale2: float = 0.02):
    """Random complex closed-shell singles ``(o,v)`` and doubles ``(o,o,v,v)``.

    The doubles obey the closed-shell pair symmetry ``x[i,j,a,b] = x[j,i,b,a]``.
    """
    x1 = scale1 * (rng.normal(size=(o, v)) + 1j * rng.normal(size=(o, v)))
    x2 = scale2 * (rng.normal(size=(o, o, v, v)) + 1j * rng.normal(size=(o, o, v, v)))
    x2 = 0.5 * (x2 + x2.transpose(1, 0, 3, 2))
    return x1, x2


def random_state(o: int, v: int, seed: int, scale1: float = 0.05, scale2: float = 0.02):
    """A random non-stationary complex state ``(t1, t2, l1, l2)`` in closed-shell variables."""
    rng = np.random.default_rng(seed)
    t1, t2 = random_amplitudes(o, v, rng, scale1, scale2)
    l1, l2 = random_amplitudes(o, v, rng, scale1, scale2)
    return t1, t2, l1, l2


def pack_state(t1, t2, l1, l2) -> np.ndarray:
    """Concatenate ``[T1 | T2 | L1 | L2]`` (each row-major) into one complex128 vector."""
    return np.concatenate([np.ravel(t1), np.ravel(t2), np.ravel(l1), np.ravel(l2)]).astype(np.complex128)


def unpack_state(y: np.ndarray, o: int, v: int):
    """Split a packed ``[T1 | T2 | L1 | L2]`` vector back into its four arrays."""
    n1, n2 = o * v, o * o * v * v
    y = np.asarray(y)
    return (y[:n1].reshape(o, v), y[n1:n1 + n2].reshape(o, o, v, v),
            y[n1 + n2:2 * n1 + n2].reshape(o, v), y[2 * n1 + n2:].reshape(o, o, v, v))


def state_size(o: int, v: int) -> int:
    """Number of complex entries in the packed state."""
    return 2 * (o * v + o * o * v * v)
