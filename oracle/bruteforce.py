"""Brute-force determinant-space evaluation of the RT-CC definitions (pins the factorised oracle).

Oracle (test infrastructure). Everything here is the plain definition, evaluated
with second-quantised operators acting on the full N-electron determinant space
of a tiny spin-orbital system:

* R_T,mu  = <mu| e^{-T} H e^{T} |0>                        (Eq. derivT, Eq. simtranH)
* R_L,mu  = <0|(1+Lambda) e^{-T} (H tau_mu - tau_mu H) e^{T} |0>   (Eq. derivL;
  tau_mu commutes with T, so [Hbar, tau_mu] = e^{-T}[H, tau_mu]e^{T})
* mu_a    = <0|(1+Lambda) e^{-T} mu_a e^{T} |0>               (Eq. dipole)
* E       = <0| e^{-T} H e^{T} |0> - <0|H|0>

with H = sum_pq h_pq p^+ q + 1/4 sum <pq||rs> p^+ q^+ s r and the core matrix
h = f - sum_k <pk||qk> chosen so that the normal-ordered Fock operator is f.
The exponentials are the terminating Taylor series (T is nilpotent).

Determinants are bit strings over the spin orbitals in the order used by
``spinorb`` (occupied first), |D> = a+_{k1} a+_{k2} ... |vac> with k1 < k2 < ...
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


class DeterminantSpace:
    def __init__(self, nso: int, nel: int):
        self.nso, self.nel = nso, nel
        masks = [sum(1 << k for k in c) for c in combinations(range(nso), nel)]
        self.masks = np.array(sorted(masks), dtype=np.int64)
        self.dim = self.masks.size
        self.ref = int(np.searchsorted(self.masks, (1 << nel) - 1))
        self._E = {}

    def E(self, p: int, q: int) -> sp.csr_matrix:
        """Sparse matrix of the excitation operator p^+ q."""
        key = (p, q)
        if key in self._E:
            return self._E[key]
        m = self.masks
        has_q = (m >> q) & 1 == 1
        m1 = m & ~(1 << q)
        ok = has_q & (((m1 >> p) & 1) == 0)
        src = np.nonzero(ok)[0]
        m1 = m1[src]
        s_q = np.bitwise_count(m[src] & ((1 << q) - 1)) & 1
        s_p = np.bitwise_count(m1 & ((1 << p) - 1)) & 1
        dst_mask = m1 | (1 << p)
        dst = np.searchsorted(self.masks, dst_mask)
        sign = np.where((s_q + s_p) % 2 == 0, 1.0, -1.0)
        mat = sp.csr_matrix((sign, (dst, src)), shape=(self.dim, self.dim))
        self._E[key] = mat
        return mat

    def vac(self) -> np.ndarray:
        x = np.zeros(self.dim, dtype=np.complex128)
        x[self.ref] = 1.0
        return x


def _apply_hamiltonian(space, h, g, x, transpose=False):
    """H x (or H^T x) without building H: one-body via E_pq, two-body via E_pr E_qs - delta_qr E_ps."""
    M = space.nso
    out = np.zeros_like(x)
    hh = h.T if transpose else h
    for p in range(M):
        for q in range(M):
            if hh[p, q] != 0:
                out += hh[p, q] * (space.E(p, q) @ x)
    if g is None:
        return out
    # 1/4 sum g[p,q,r,s] p+ q+ s r ;  p+ q+ s r = E_pr E_qs - delta_qr E_ps
    # transpose: (E_pr E_qs)^T = E_sq E_rp ; E_ps^T = E_sp
    Y = np.stack([space.E(q, s) @ x if not transpose else space.E(s, q) @ x
                  for q in range(M) for s in range(M)])  # index (q,s)
    if not transpose:
        Z = np.einsum("pqrs,qsx->prx", g, Y.reshape(M, M, -1))
        for p in range(M):
            for r in range(M):
                out += 0.25 * (space.E(p, r) @ Z[p, r])
        c = np.einsum("pqqs->ps", g)
        for p in range(M):
            for s in range(M):
                if c[p, s] != 0:
                    out -= 0.25 * c[p, s] * (space.E(p, s) @ x)
    else:
        # sum g[p,q,r,s] E_sq E_rp x : first W[p,r] = E_rp x, then E_sq applied
        W = np.stack([space.E(r, p) @ x for p in range(M) for r in range(M)]).reshape(M, M, -1)
        Z = np.einsum("pqrs,prx->qsx", g, W)
        for q in range(M):
            for s in range(M):
                out += 0.25 * (space.E(s, q) @ Z[q, s])
        c = np.einsum("pqqs->ps", g)
        for p in range(M):
            for s in range(M):
                if c[p, s] != 0:
                    out -= 0.25 * c[p, s] * (space.E(s, p) @ x)
    return out


class BruteForce:
    """Determinant-space evaluator for a spin-orbital system with ``nocc`` occupied spin orbitals."""

    def __init__(self, f, g, nocc):
        self.f, self.g, self.no = f, g, nocc
        M = f.shape[0]
        self.nv = M - nocc
        self.space = DeterminantSpace(M, nocc)
        core = np.einsum("pkqk->pq", g[:, :nocc, :, :nocc]) if g is not None else 0.0
        self.h = f - core

    # -- excitation operators -------------------------------------------------
    def _occ(self):
        return range(self.no)

    def _vir(self):
        return range(self.no, self.no + self.nv)

    def singles(self):
        return [(i, a) for i in self._occ() for a in self._vir()]

    def doubles(self):
        occ, vir = list(self._occ()), list(self._vir())
        return [(i, j, a, b) for i, j in combinations(occ, 2) for a, b in combinations(vir, 2)]

    def tau(self, mu):
        S = self.space
        if len(mu) == 2:
            i, a = mu
            return S.E(a, i)
        i, j, a, b = mu
        return S.E(a, i) @ S.E(b, j)

    def cluster(self, X1, X2):
        """sum_ia x_ia a+ i + sum_{i<j,a<b} x_ijab a+ b+ j i (spin-orbital arrays, vir index offset removed)."""
        S = self.space
        op = sp.csr_matrix((S.dim, S.dim), dtype=np.complex128)
        for (i, a) in self.singles():
            c = X1[i, a - self.no]
            if c != 0:
                op = op + c * self.tau((i, a))
        for (i, j, a, b) in self.doubles():
            c = X2[i, j, a - self.no, b - self.no]
            if c != 0:
                op = op + c * self.tau((i, j, a, b))
        return op.tocsr()

    @staticmethod
    def _expm_apply(T, x, sign=1.0):
        out = x.copy()
        term = x.copy()
        k = 1
        while True:
            term = (sign / k) * (T @ term)
            if not np.any(term):
                break
            out += term
            k += 1
            if k > 64:
                raise RuntimeError("cluster operator is not nilpotent")
        return out

    # -- definitions ----------------------------------------------------------------
    def right(self, T1, T2):
        T = self.cluster(T1, T2)
        return T, self._expm_apply(T, self.space.vac())

    def t_residual(self, T1, T2):
        T, r = self.right(T1, T2)
        Hr = _apply_hamiltonian(self.space, self.h, self.g, r)
        x = self._expm_apply(T, Hr, -1.0)
        e0 = self.space.vac()
        R1 = np.zeros((self.no, self.nv), complex)
        R2 = np.zeros((self.no, self.no, self.nv, self.nv), complex)
        for (i, a) in self.singles():
            R1[i, a - self.no] = (self.tau((i, a)) @ e0) @ x
        for (i, j, a, b) in self.doubles():
            val = (self.tau((i, j, a, b)) @ e0) @ x
            ia, ja, aa, ba = i, j, a - self.no, b - self.no
            R2[ia, ja, aa, ba] = val
            R2[ja, ia, aa, ba] = -val
            R2[ia, ja, ba, aa] = -val
            R2[ja, ia, ba, aa] = val
        energy = e0 @ x - e0 @ _apply_hamiltonian(self.space, self.h, self.g, e0)
        return R1, R2, energy

    def left(self, T, L1, L2):
        """Column vector of the bra <0|(1+Lambda) e^{-T}."""
        e0 = self.space.vac()
        Lop = self.cluster(L1, L2)   # same coefficients, excitation form; bra = (tau e0)^T
        bra = e0 + Lop @ e0
        return self._expm_apply(T.T.tocsr(), bra, -1.0)

    def l_residual(self, T1, T2, L1, L2):
        T, r = self.right(T1, T2)
        lcol = self.left(T, L1, L2)
        Hr = _apply_hamiltonian(self.space, self.h, self.g, r)
        lH = _apply_hamiltonian(self.space, self.h, self.g, lcol, transpose=True)
        R1 = np.zeros((self.no, self.nv), complex)
        R2 = np.zeros((self.no, self.no, self.nv, self.nv), complex)
        for (i, a) in self.singles():
            tmu = self.tau((i, a))
            R1[i, a - self.no] = lH @ (tmu @ r) - lcol @ (tmu @ Hr)
        for (i, j, a, b) in self.doubles():
            tmu = self.tau((i, j, a, b))
            val = lH @ (tmu @ r) - lcol @ (tmu @ Hr)
            ia, ja, aa, ba = i, j, a - self.no, b - self.no
            R2[ia, ja, aa, ba] = val
            R2[ja, ia, aa, ba] = -val
            R2[ia, ja, ba, aa] = -val
            R2[ja, ia, ba, aa] = val
        return R1, R2

    def expectation(self, op1, T1, T2, L1, L2):
        """<0|(1+Lambda) e^{-T} O e^{T}|0> for the one-body operator O = sum o_pq p+ q."""
        T, r = self.right(T1, T2)
        lcol = self.left(T, L1, L2)
        Or = _apply_hamiltonian(self.space, op1, None, r)
        return lcol @ Or
