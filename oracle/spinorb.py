"""Spatial (closed-shell) <-> spin-orbital conversion for the oracle.

Spin-orbital ordering: ``[occ alpha (o) | occ beta (o) | vir alpha (v) | vir beta (v)]``.
Physicists' integrals ``<pq|rs> = (pr|qs) delta(s_p,s_r) delta(s_q,s_s)``, and the
antisymmetrised ``<pq||rs> = <pq|rs> - <pq|sr>``.

Closed-shell map (the paper notes that spin adaptation carries over from the
ground-state theory; Theory, "Propagation of the RT-CC equations"):
``x_i^a = x_{ia}^{aa}`` (both spins), ``x_ij^ab = x_{i alpha, j beta}^{a alpha, b beta}``,
same-spin doubles ``x_ij^ab - x_ij^ba``. T and Lambda use the same map.
"""
from __future__ import annotations

import numpy as np


def so_index(o: int, v: int):
    """Return (spatial index, spin) arrays for the 2n spin orbitals."""
    n = o + v
    spatial = np.concatenate([np.arange(o), np.arange(o), o + np.arange(v), o + np.arange(v)])
    spin = np.concatenate([np.zeros(o, int), np.ones(o, int), np.zeros(v, int), np.ones(v, int)])
    assert spatial.size == 2 * n
    return spatial, spin


def so_one_body(h: np.ndarray, o: int, v: int) -> np.ndarray:
    """Spin-orbital matrix ``h_PQ = h_pq delta(s_P, s_Q)`` of a spatial one-body operator."""
    sp, s = so_index(o, v)
    return h[np.ix_(sp, sp)] * (s[:, None] == s[None, :])


def so_antisym_eri(eri: np.ndarray, o: int, v: int) -> np.ndarray:
    """``<PQ||RS>`` from chemists' spatial ``(pq|rs)``."""
    sp, s = so_index(o, v)
    phys = eri.transpose(0, 2, 1, 3)  # <pq|rs> = (pr|qs)
    g = phys[np.ix_(sp, sp, sp, sp)]
    d_pr = (s[:, None] == s[None, :])[:, None, :, None]
    d_qs = (s[:, None] == s[None, :])[None, :, None, :]
    direct = g * (d_pr & d_qs)
    return direct - direct.transpose(0, 1, 3, 2)


def cs_to_so(x1: np.ndarray, x2: np.ndarray):
    """Closed-shell singles/doubles -> spin-orbital arrays (O=2o, V=2v)."""
    o, v = x1.shape
    X1 = np.zeros((2 * o, 2 * v), dtype=np.result_type(x1, x2, np.complex128))
    X1[:o, :v] = x1
    X1[o:, v:] = x1
    X2 = np.zeros((2 * o, 2 * o, 2 * v, 2 * v), dtype=X1.dtype)
    a, b = slice(0, o), slice(o, 2 * o)   # occupied alpha / beta
    A, B = slice(0, v), slice(v, 2 * v)   # virtual alpha / beta
    xT = x2.transpose(0, 1, 3, 2)          # x_ij^ba
    same = x2 - xT
    X2[a, a, A, A] = same
    X2[b, b, B, B] = same
    X2[a, b, A, B] = x2
    X2[a, b, B, A] = -xT
    X2[b, a, B, A] = x2
    X2[b, a, A, B] = -xT
    return X1, X2


def so_to_cs(X1: np.ndarray, X2: np.ndarray, o: int, v: int):
    """Spin-orbital singles/doubles -> closed-shell components (alpha; alpha-beta)."""
    return X1[:o, :v].copy(), X2[:o, o:, :v, v:].copy()
