"""Spin-orbital CCSD and Lambda-CCSD residuals, the RT-CC right-hand side and the dipole.

Oracle (test infrastructure; see the package docstring). Plain complex128 NumPy,
spin orbitals, full (non-canonical, field-dressed) Fock matrix.

Definitions followed (paper, Theory section):

* Eq. derivT:  <mu| Hbar |0> = i dt_mu/dt, i.e. dt/dt = -i R_T with
  R_T,mu = <mu| e^{-T} H e^{T} |0>.
* Eq. derivL:  <0|(1+Lambda)[Hbar, tau_mu]|0> = -i dlambda_mu/dt, i.e.
  dlambda/dt = +i R_L with R_L,mu = <0|(1+Lambda)[Hbar, tau_mu]|0>.
* Eq. simtranH: Hbar = e^{-T} H e^{T}.
* The field enters only through the Fock matrix, f(t) = f - sum_a E_a(t) mu_a
  (dipole coupling V(t) = -mu E(t), linear-absorption subsection); the
  two-electron integrals do not change (orbitals are kept frozen).

The paper does not print the working equations ("simply the residual
equations" of ground-state CC). The oracle evaluates the definitions through
the factorised spin-orbital CCSD equations of Stanton and Gauss (T) and the
Lambda equations of Gauss and Stanton, with every Fock term kept (no
orbital-energy denominators), which are exact for singles and doubles; the
module ``bruteforce`` pins each of them against the determinant-space
definitions at random non-stationary amplitudes.

Index convention: ``g[p,q,r,s] = <pq||rs>``; occupied i,j,m,n; virtual
a,b,e,f. ``P(pq) X = X - X(p<->q)``.
"""
from __future__ import annotations

from functools import partial

import numpy as np

from . import spinorb

_einsum = partial(np.einsum, optimize=True)  # BLAS-backed pairwise contraction


def _blocks(g, no):
    """Named views of the antisymmetrised integrals (``o`` = occupied, ``v`` = virtual)."""
    o, v = slice(0, no), slice(no, g.shape[0])
    names = {}
    for key in ("oooo", "ooov", "oovo", "oovv", "ovoo", "ovov", "ovvo", "ovvv",
                "vovv", "vvvo", "vvvv", "vooo", "vovo", "voov", "vvoo", "vvov"):
        sl = tuple(o if c == "o" else v for c in key)
        names[key] = g[sl]
    return names


def _Pij(x):
    return x - x.swapaxes(0, 1)


def _Pab(x):
    return x - x.swapaxes(2, 3)


def taus(t1, t2):
    """tau-tilde and tau of the factorised equations."""
    tt = _einsum("ia,jb->ijab", t1, t1)
    tt = tt - tt.swapaxes(2, 3)
    return t2 + 0.5 * tt, t2 + tt


def intermediates(f, g, t1, t2):
    """One-body F and two-body W intermediates of the Stanton-Gauss CCSD equations.

    ``g`` may be ``None`` (a purely one-body operator); then every term that
    carries a two-electron integral is omitted.
    """
    no = t1.shape[0]
    o, v = slice(0, no), slice(no, f.shape[0])
    fov, foo, fvv = f[o, v], f[o, o], f[v, v]
    tau_t, tau = taus(t1, t2)
    Fae = fvv - 0.5 * _einsum("me,ma->ae", fov, t1)
    Fmi = foo + 0.5 * _einsum("ie,me->mi", t1, fov)
    Fme = fov.astype(np.complex128)
    W = {}
    if g is not None:
        b = _blocks(g, no)
        Fae = Fae + _einsum("mf,mafe->ae", t1, b["ovvv"]) - 0.5 * _einsum("mnaf,mnef->ae", tau_t, b["oovv"])
        Fmi = Fmi + _einsum("ne,mnie->mi", t1, b["ooov"]) + 0.5 * _einsum("inef,mnef->mi", tau_t, b["oovv"])
        Fme = Fme + _einsum("nf,mnef->me", t1, b["oovv"])
        x = _einsum("je,mnie->mnij", t1, b["ooov"])
        W["mnij"] = b["oooo"] + x - x.swapaxes(2, 3) + 0.25 * _einsum("ijef,mnef->mnij", tau, b["oovv"])
        x = _einsum("mb,amef->abef", t1, b["vovv"])
        W["abef"] = b["vvvv"] - (x - x.swapaxes(0, 1)) + 0.25 * _einsum("mnab,mnef->abef", tau, b["oovv"])
        W["mbej"] = (b["ovvo"] + _einsum("jf,mbef->mbej", t1, b["ovvv"])
                     - _einsum("nb,mnej->mbej", t1, b["oovo"])
                     - _einsum("jnfb,mnef->mbej", 0.5 * t2 + _einsum("jf,nb->jnfb", t1, t1), b["oovv"]))
    return Fae, Fmi, Fme, W


def t_residual(f, g, t1, t2):
    """R_T = <mu|e^{-T} H e^{T}|0> for singles and doubles (Eq. derivT's left side)."""
    no = t1.shape[0]
    o, v = slice(0, no), slice(no, f.shape[0])
    fov = f[o, v]
    tau_t, tau = taus(t1, t2)
    Fae, Fmi, Fme, W = intermediates(f, g, t1, t2)

    r1 = (fov + _einsum("ie,ae->ia", t1, Fae) - _einsum("ma,mi->ia", t1, Fmi)
          + _einsum("imae,me->ia", t2, Fme))
    X = Fae - 0.5 * _einsum("mb,me->be", t1, Fme)
    Y = Fmi + 0.5 * _einsum("je,me->mj", t1, Fme)
    r2 = _Pab(_einsum("ijae,be->ijab", t2, X)) - _Pij(_einsum("imab,mj->ijab", t2, Y))
    if g is not None:
        b = _blocks(g, no)
        r1 = r1 - _einsum("nf,naif->ia", t1, b["ovov"]) \
            - 0.5 * _einsum("imef,maef->ia", t2, b["ovvv"]) \
            - 0.5 * _einsum("mnae,nmei->ia", t2, b["oovo"])
        r2 = r2 + b["oovv"]
        r2 = r2 + 0.5 * _einsum("mnab,mnij->ijab", tau, W["mnij"])
        r2 = r2 + 0.5 * _einsum("ijef,abef->ijab", tau, W["abef"])
        x = _einsum("imae,mbej->ijab", t2, W["mbej"]) - _einsum("ie,ma,mbej->ijab", t1, t1, b["ovvo"])
        r2 = r2 + _Pab(_Pij(x))
        r2 = r2 + _Pij(_einsum("ie,abej->ijab", t1, b["vvvo"]))
        r2 = r2 - _Pab(_einsum("ma,mbij->ijab", t1, b["ovoo"]))
    return r1, r2


def energy(f, g, t1, t2):
    """Correlation part of <0|Hbar|0>: sum f_ia t_ia + 1/4 <ij||ab> t_ijab + 1/2 <ij||ab> t_ia t_jb."""
    no = t1.shape[0]
    o, v = slice(0, no), slice(no, f.shape[0])
    e = _einsum("ia,ia->", f[o, v], t1)
    if g is not None:
        govv = g[o, o, v, v]
        e = e + 0.25 * _einsum("ijab,ijab->", govv, t2) + 0.5 * _einsum("ijab,ia,jb->", govv, t1, t1)
    return e


def hbar(f, g, t1, t2):
    """Elements of Hbar used by the Lambda equations (Gauss-Stanton factorisation)."""
    no = t1.shape[0]
    _, tau = taus(t1, t2)
    Fae, Fmi, Fme, W = intermediates(f, g, t1, t2)
    H = {"ov": Fme,
         "oo": Fmi + 0.5 * _einsum("ie,me->mi", t1, Fme),
         "vv": Fae - 0.5 * _einsum("ma,me->ae", t1, Fme)}
    if g is None:
        # the Fock parts of Hbar_mbij and Hbar_abei survive without two-electron integrals
        H["ovoo"] = -_einsum("me,ijbe->mbij", Fme, t2)
        H["vvvo"] = -_einsum("me,miab->abei", Fme, t2)
        return H
    b = _blocks(g, no)
    H["oooo"] = W["mnij"] + 0.25 * _einsum("ijef,mnef->mnij", tau, b["oovv"])
    H["vvvv"] = W["abef"] + 0.25 * _einsum("mnab,mnef->abef", tau, b["oovv"])
    H["ovvo"] = W["mbej"] - 0.5 * _einsum("jnfb,mnef->mbej", t2, b["oovv"])
    H["ooov"] = b["ooov"] + _einsum("if,mnfe->mnie", t1, b["oovv"])
    H["vovv"] = b["vovv"] - _einsum("na,nmef->amef", t1, b["oovv"])
    x = b["ovvo"] - _einsum("njbf,mnef->mbej", t2, b["oovv"])
    H["ovoo"] = (b["ovoo"] - _einsum("me,ijbe->mbij", Fme, t2)
                 - _einsum("nb,mnij->mbij", t1, H["oooo"])
                 + 0.5 * _einsum("mbef,ijef->mbij", b["ovvv"], tau)
                 + _Pab(_einsum("mnie,jnbe->mbij", b["ooov"], t2))
                 + _Pab(_einsum("ie,mbej->mbij", t1, x)))
    x = b["ovvo"] - _einsum("nibf,mnef->mbei", t2, b["oovv"])
    y = _einsum("mbef,miaf->abei", b["ovvv"], t2) + _einsum("ma,mbei->abei", t1, x)
    H["vvvo"] = (b["vvvo"] - _einsum("me,miab->abei", Fme, t2)
                 + _einsum("if,abef->abei", t1, H["vvvv"])
                 + 0.5 * _einsum("mnei,mnab->abei", b["oovo"], tau)
                 - (y - y.swapaxes(0, 1)))
    return H


def l_residual(f, g, t1, t2, l1, l2):
    """R_L = <0|(1+Lambda)[Hbar, tau_mu]|0> (Eq. derivL's left side), singles and doubles."""
    H = hbar(f, g, t1, t2)
    no = t1.shape[0]
    r1 = (H["ov"] + _einsum("ie,ea->ia", l1, H["vv"]) - _einsum("ma,im->ia", l1, H["oo"])
          + 0.5 * _einsum("imef,efam->ia", l2, H["vvvo"])
          - 0.5 * _einsum("mnae,iemn->ia", l2, H["ovoo"]))
    r2 = (_Pab(_einsum("ijae,eb->ijab", l2, H["vv"])) - _Pij(_einsum("imab,jm->ijab", l2, H["oo"]))
          + _Pij(_Pab(_einsum("ia,jb->ijab", l1, H["ov"]))))
    if g is not None:
        o, v = slice(0, no), slice(no, f.shape[0])
        govv = g[o, o, v, v]
        Gvv = -0.5 * _einsum("mnef,mnaf->ae", t2, l2)
        Goo = 0.5 * _einsum("mnef,inef->mi", t2, l2)
        r1 = r1 + (_einsum("me,ieam->ia", l1, H["ovvo"])
                   - _einsum("ef,eifa->ia", Gvv, H["vovv"])
                   - _einsum("mn,mina->ia", Goo, H["ooov"]))
        r2 = r2 + (govv
                   + 0.5 * _einsum("mnab,ijmn->ijab", l2, H["oooo"])
                   + 0.5 * _einsum("ijef,efab->ijab", l2, H["vvvv"])
                   + _Pij(_einsum("ie,ejab->ijab", l1, H["vovv"]))
                   - _Pab(_einsum("ma,ijmb->ijab", l1, H["ooov"]))
                   + _Pij(_Pab(_einsum("imae,jebm->ijab", l2, H["ovvo"])))
                   + _Pab(_einsum("ijae,be->ijab", govv, Gvv))
                   - _Pij(_einsum("imab,mj->ijab", govv, Goo)))
    return r1, r2


class SpinOrbitalSystem:
    """Spin-orbital Fock, antisymmetrised integrals and dipole integrals of a closed-shell system."""

    def __init__(self, eri, fock, mu, o, v):
        """``eri=None`` builds a system without two-electron integrals (enough for the dipole)."""
        self.o, self.v = o, v
        self.f0 = spinorb.so_one_body(np.asarray(fock, float), o, v)
        self.g = None if eri is None else spinorb.so_antisym_eri(np.asarray(eri, float), o, v)
        self.mu = np.stack([spinorb.so_one_body(np.asarray(m, float), o, v) for m in mu])
        self.mu_ref = np.array([np.trace(m[:2 * o, :2 * o]) for m in self.mu])

    def fock(self, E):
        """f(t) = f - sum_a E_a mu_a (field-dressed Fock matrix)."""
        E = np.asarray(E, float)
        return self.f0 - _einsum("a,apq->pq", E, self.mu)


def _so_amps(t1, t2, l1, l2):
    T1, T2 = spinorb.cs_to_so(t1, t2)
    L1, L2 = spinorb.cs_to_so(l1, l2)
    return T1, T2, L1, L2


def rhs(sys: SpinOrbitalSystem, t1, t2, l1, l2, E):
    """Closed-shell components of (dt/dt, dlambda/dt) = (-i R_T, +i R_L) at field E (3-vector)."""
    o, v = sys.o, sys.v
    T1, T2, L1, L2 = _so_amps(t1, t2, l1, l2)
    f = sys.fock(E)
    rt1, rt2 = t_residual(f, sys.g, T1, T2)
    rl1, rl2 = l_residual(f, sys.g, T1, T2, L1, L2)
    rt1, rt2 = spinorb.so_to_cs(rt1, rt2, o, v)
    rl1, rl2 = spinorb.so_to_cs(rl1, rl2, o, v)
    return -1j * rt1, -1j * rt2, 1j * rl1, 1j * rl2


def residuals(sys: SpinOrbitalSystem, t1, t2, l1, l2, E=(0.0, 0.0, 0.0)):
    """Closed-shell components of (R_T1, R_T2, R_L1, R_L2)."""
    o, v = sys.o, sys.v
    T1, T2, L1, L2 = _so_amps(t1, t2, l1, l2)
    f = sys.fock(E)
    rt = spinorb.so_to_cs(*t_residual(f, sys.g, T1, T2), o, v)
    rl = spinorb.so_to_cs(*l_residual(f, sys.g, T1, T2, L1, L2), o, v)
    return rt[0], rt[1], rl[0], rl[1]


def one_body_rhs(sys: SpinOrbitalSystem, t1, t2, l1, l2, n):
    """RHS of the operator sum_a n_a mu_a alone (no two-electron part): (-i R_T[mu,0], +i R_L[mu,0])."""
    o, v = sys.o, sys.v
    T1, T2, L1, L2 = _so_amps(t1, t2, l1, l2)
    m = _einsum("a,apq->pq", np.asarray(n, float), sys.mu)
    rt1, rt2 = spinorb.so_to_cs(*t_residual(m, None, T1, T2), o, v)
    rl1, rl2 = spinorb.so_to_cs(*l_residual(m, None, T1, T2, L1, L2), o, v)
    return -1j * rt1, -1j * rt2, 1j * rl1, 1j * rl2


def lagrangian(f, g, T1, T2, L1, L2):
    """L = <0|(1+Lambda) Hbar |0> minus the reference energy (spin-orbital amplitudes)."""
    r1, r2 = t_residual(f, g, T1, T2)
    return energy(f, g, T1, T2) + np.sum(L1 * r1) + 0.25 * np.sum(L2 * r2)


def dipole(sys: SpinOrbitalSystem, t1, t2, l1, l2):
    """mu_a = <0|(1+Lambda) e^{-T} mu_a e^{T}|0> (Eq. dipole), complex, reference part included.

    Because the Lagrangian is linear in the Hamiltonian, the expectation value
    of a one-body operator equals its reference value plus the Lagrangian
    evaluated with that operator as the "Fock matrix" and no two-electron part.
    """
    T1, T2, L1, L2 = _so_amps(t1, t2, l1, l2)
    return np.array([sys.mu_ref[a] + lagrangian(sys.mu[a], None, T1, T2, L1, L2) for a in range(3)])
