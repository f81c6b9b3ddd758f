"""MI355X real-time CCSD propagation: thin Python binding of the HIP library ``librtcc.so``.

Argument marshalling only: every step of the right-hand side, the integrators,
the kick, the dipole and the ground state runs in the library's HIP kernels
(see ``include/rtcc.h``). PyTorch provides device memory and the stream. There
is no CPU fallback: if the library is missing, importing ``RTCC`` fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtcc.so")
TUNING_PATH = os.path.join(_HERE, "tuned_gemm.txt")

FP64, FP32, BF16X3 = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
FIELD_NONE, FIELD_GAUSSIAN, FIELD_KICK = 0, 1, 2


class Field(ctypes.Structure):
    """rtcc_field: kind, E0, omega, sigma, t0, n[3]."""
    _fields_ = [("kind", ctypes.c_int), ("E0", ctypes.c_double), ("omega", ctypes.c_double),
                ("sigma", ctypes.c_double), ("t0", ctypes.c_double), ("n", ctypes.c_double * 3)]

    @classmethod
    def gaussian(cls, E0, omega, sigma, t0, n):
        return cls(FIELD_GAUSSIAN, E0, omega, sigma, t0, (ctypes.c_double * 3)(*n))

    @classmethod
    def none(cls):
        return cls(FIELD_NONE, 0.0, 0.0, 1.0, 0.0, (ctypes.c_double * 3)(0.0, 0.0, 0.0))


MAX_STAGES = 6
TAB_RK4, TAB_CASHKARP, TAB_RKF45, TAB_GL2, TAB_GL3 = 1, 2, 3, 4, 5
_TAB = {"rk4": TAB_RK4, "cashkarp": TAB_CASHKARP, "rkf45": TAB_RKF45, "gl2": TAB_GL2, "gl3": TAB_GL3}


class Tableau(ctypes.Structure):
    """rtcc_tableau: stages, err_order, a[6][6], b[6], b_err[6], c[6]."""
    _fields_ = [("stages", ctypes.c_int), ("err_order", ctypes.c_int),
                ("a", (ctypes.c_double * MAX_STAGES) * MAX_STAGES), ("b", ctypes.c_double * MAX_STAGES),
                ("b_err", ctypes.c_double * MAX_STAGES), ("c", ctypes.c_double * MAX_STAGES)]

    @classmethod
    def builtin(cls, name):
        """One of the library's tableaux: "rk4", "cashkarp", "rkf45", "gl2", "gl3" (rtcc_tableau_builtin)."""
        L = load_library()
        t = cls()
        rc = L.rtcc_tableau_builtin(_TAB[name] if isinstance(name, str) else int(name), ctypes.byref(t))
        if rc != 0:
            raise RTCCError(rc, L.rtcc_last_error(None).decode())
        return t

    @classmethod
    def from_arrays(cls, a, b, c, b_err=None, err_order=0):
        """A caller's tableau from nested sequences (a: s x s)."""
        s = len(b)
        t = cls()
        t.stages, t.err_order = s, int(err_order)
        for i in range(s):
            t.b[i], t.c[i] = float(b[i]), float(c[i])
            if b_err is not None:
                t.b_err[i] = float(b_err[i])
            for j in range(s):
                t.a[i][j] = float(a[i][j]) if j < len(a[i]) else 0.0
        return t

    def arrays(self):
        s = self.stages
        A = np.array([[self.a[i][j] for j in range(s)] for i in range(s)])
        return A, np.array(self.b[:s]), np.array(self.c[:s]), np.array(self.b_err[:s])


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librtcc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2205_05175_amd.build` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, d, i, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    L.rtcc_init.argtypes = [ctypes.POINTER(vp), i, i, dp, dp, dp, i, vp]
    L.rtcc_set_precision.argtypes = [vp, i]
    L.rtcc_rhs.argtypes = [vp, vp, d, dp, vp]
    L.rtcc_step_rk4.argtypes = [vp, vp, d, d, ctypes.POINTER(Field)]
    L.rtcc_propagate_rk4.argtypes = [vp, vp, d, d, i, ctypes.POINTER(Field), vp]
    L.rtcc_propagate_batch.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(vp),
                                       ctypes.POINTER(Field), d, d, i, ctypes.POINTER(vp)]
    L.rtcc_rhs_vjp.argtypes = [vp, vp, d, dp, vp, vp, dp]
    L.rtcc_dipole_vjp.argtypes = [vp, vp, dp, vp]
    L.rtcc_step_rk4_vjp.argtypes = [vp, vp, d, d, ctypes.POINTER(Field), vp, dp]
    L.rtcc_step_cashkarp.argtypes = [vp, vp, dp, dp, d, ctypes.POINTER(Field), ctypes.POINTER(i), dp]
    L.rtcc_set_guard.argtypes = [vp, d, i]
    L.rtcc_gemm.argtypes = [i, i64, i64, i64, d, vp, vp, i64, i, vp, vp, i64, i, d, vp, vp, i64,
                            ctypes.POINTER(i), i, ctypes.POINTER(ctypes.c_float), vp]
    L.rtcc_load_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(i)]
    L.rtcc_check_state_noalloc.argtypes = [i, i, vp, vp, vp]
    L.rtcc_peak_probe.argtypes = [i, i64, dp]
    L.rtcc_mixed_schedule.argtypes = [d, d, d, d, ctypes.POINTER(Field), i, dp, ctypes.POINTER(i)]
    L.rtcc_propagate_rk4_mixed.argtypes = [vp, vp, d, d, d, d, ctypes.POINTER(Field), vp, vp]
    L.rtcc_propagate_cashkarp.argtypes = [vp, vp, d, d, d, d, ctypes.POINTER(Field), i, i, dp, dp,
                                          ctypes.POINTER(i), ctypes.POINTER(i), dp]
    tp = ctypes.POINTER(Tableau)
    L.rtcc_tableau_builtin.argtypes = [i, tp]
    L.rtcc_step_tableau.argtypes = [vp, vp, d, d, tp, ctypes.POINTER(Field), d, i, dp, ctypes.POINTER(i)]
    L.rtcc_propagate_embedded.argtypes = [vp, vp, d, d, d, d, tp, ctypes.POINTER(Field), i, i, dp, dp,
                                          ctypes.POINTER(i), ctypes.POINTER(i), dp]
    L.rtcc_dipole.argtypes = [vp, vp, dp]
    L.rtcc_dipole_dev.argtypes = [vp, vp, vp]
    L.rtcc_ground_state.argtypes = [vp, vp, d, i, dp]
    L.rtcc_kick.argtypes = [vp, vp, d, dp]
    L.rtcc_check_state.argtypes = [vp, vp, ctypes.POINTER(i64)]
    L.rtcc_info.argtypes = [vp, ctypes.POINTER(i64)]
    L.rtcc_profile.argtypes = [vp, i]
    L.rtcc_profile_read.argtypes = [vp, ctypes.POINTER(i64), dp, dp, dp]
    L.rtcc_destroy.argtypes = [vp]
    L.rtcc_destroy.restype = None
    L.rtcc_last_error.argtypes = [vp]
    L.rtcc_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("rtcc_destroy", "rtcc_last_error"):
            getattr(L, name).restype = ctypes.c_int
    # the GEMM tuning table written by autotune.py (RTCC_NO_TUNING=1: the library's own rules only)
    if os.path.exists(TUNING_PATH) and os.environ.get("RTCC_NO_TUNING", "0") != "1":
        n = ctypes.c_int(0)
        if L.rtcc_load_tuning(TUNING_PATH.encode(), ctypes.byref(n)) != 0:
            raise RTCCError(-1, L.rtcc_last_error(None).decode())
    _lib = L
    return L


EXPORTED = ("rtcc_init", "rtcc_set_precision", "rtcc_rhs", "rtcc_step_rk4", "rtcc_propagate_rk4",
            "rtcc_propagate_batch", "rtcc_rhs_vjp", "rtcc_dipole_vjp", "rtcc_step_rk4_vjp", "rtcc_step_cashkarp",
            "rtcc_set_guard", "rtcc_mixed_schedule", "rtcc_propagate_rk4_mixed", "rtcc_propagate_cashkarp",
            "rtcc_gemm", "rtcc_load_tuning", "rtcc_check_state_noalloc", "rtcc_peak_probe", "rtcc_tableau_builtin",
            "rtcc_step_tableau", "rtcc_propagate_embedded",
            "rtcc_dipole", "rtcc_dipole_dev", "rtcc_ground_state", "rtcc_kick", "rtcc_check_state", "rtcc_info",
            "rtcc_profile", "rtcc_profile_read", "rtcc_destroy", "rtcc_last_error")


class RTCCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtcc error {code}: {msg}")
        self.code = code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class RTCC:
    """One closed-shell system on one GPU (a context of the C ABI).

    ``eri`` (n^4, chemists' order), ``fock`` (n x n) and ``mu`` (3 x n x n) are host float64
    arrays; states are complex128 CUDA tensors of length ``state_size(o, v)`` laid out as
    [T1 | T2 | L1 | L2].
    """

    def __init__(self, eri, fock, mu, o, v, precision="fp64", stream=None):
        import torch
        self.L = load_library()
        self.o, self.v = int(o), int(v)
        self.n = self.o + self.v
        self.nstate = 2 * (self.o * self.v + (self.o * self.v) ** 2)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        fock = np.ascontiguousarray(fock, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        n = self.n
        if eri.shape != (n, n, n, n) or fock.shape != (n, n) or mu.shape != (3, n, n):
            raise ValueError("integral shapes do not match o + v")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = ctypes.c_void_p()
        rc = self.L.rtcc_init(ctypes.byref(self.ctx), self.o, self.v, _dptr(eri), _dptr(fock), _dptr(mu),
                              _PREC[precision], ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise RTCCError(rc, self.L.rtcc_last_error(None).decode())

    # -- helpers ---------------------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise RTCCError(rc, self.L.rtcc_last_error(self.ctx).decode())

    def _state(self, y, name="y"):
        import torch
        if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.complex128
                and y.is_contiguous() and y.numel() == self.nstate):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of {self.nstate} entries")
        return ctypes.c_void_p(y.data_ptr())

    def new_state(self):
        import torch
        return torch.zeros(self.nstate, dtype=torch.complex128, device="cuda")

    # -- ABI -------------------------------------------------------------------------------
    def set_precision(self, precision):
        self._check(self.L.rtcc_set_precision(self.ctx, _PREC[precision]))

    def rhs(self, y, E, out=None, t=0.0):
        if out is None:
            out = self.new_state()
        Ea = (ctypes.c_double * 3)(*[float(x) for x in E])
        self._check(self.L.rtcc_rhs(self.ctx, self._state(y), float(t), Ea, self._state(out, "out")))
        return out

    def step_rk4(self, y, t, h, field=None):
        f = field if field is not None else Field.none()
        self._check(self.L.rtcc_step_rk4(self.ctx, self._state(y), float(t), float(h), ctypes.byref(f)))

    def propagate_rk4(self, y, t0, h, nsteps, field=None, mu_out=None):
        """nsteps RK4 steps; if mu_out (float64 CUDA tensor (nsteps+1, 6)) is given, the dipole is recorded."""
        import torch
        f = field if field is not None else Field.none()
        ptr = None
        if mu_out is not None:
            if not (mu_out.is_cuda and mu_out.dtype == torch.float64 and mu_out.is_contiguous()
                    and mu_out.numel() >= 6 * (nsteps + 1)):
                raise ValueError("mu_out must be a contiguous float64 CUDA tensor with (nsteps+1)*6 entries")
            ptr = ctypes.c_void_p(mu_out.data_ptr())
        self._check(self.L.rtcc_propagate_rk4(self.ctx, self._state(y), float(t0), float(h), int(nsteps),
                                              ctypes.byref(f), ptr))

    def step_cashkarp(self, y, t, h, eps, field=None):
        f = field if field is not None else Field.none()
        tt, hh = ctypes.c_double(t), ctypes.c_double(h)
        acc, delta = ctypes.c_int(0), ctypes.c_double(0.0)
        self._check(self.L.rtcc_step_cashkarp(self.ctx, self._state(y), ctypes.byref(tt), ctypes.byref(hh),
                                              float(eps), ctypes.byref(f), ctypes.byref(acc), ctypes.byref(delta)))
        return tt.value, hh.value, bool(acc.value), delta.value

    def set_guard(self, t2_limit, check_every=50):
        """Divergence guard of the RK4 propagations (t2_limit <= 0: off)."""
        self._check(self.L.rtcc_set_guard(self.ctx, float(t2_limit), int(check_every)))

    def mixed_schedule(self, t0, t_end, h1, h2, field=None):
        """Times (t0 and every step end) of the mixed step-size RK4 schedule."""
        return mixed_schedule(t0, t_end, h1, h2, field)

    def propagate_rk4_mixed(self, y, t0, t_end, h1, h2, field=None, mu_out=None, t2norm_out=None):
        """Mixed step-size RK4 (h1 while the pulse is on, h2 elsewhere); optional dipole (nsteps+1, 6)
        and |T2| (nsteps+1) records as float64 CUDA tensors. Returns the number of steps."""
        import torch
        f = field if field is not None else Field.none()
        ns = len(mixed_schedule(t0, t_end, h1, h2, f)) - 1
        ptrs = []
        for arr, k in ((mu_out, 6), (t2norm_out, 1)):
            if arr is None:
                ptrs.append(None)
                continue
            if not (arr.is_cuda and arr.dtype == torch.float64 and arr.is_contiguous() and arr.numel() >= k * (ns + 1)):
                raise ValueError(f"record tensor must be a contiguous float64 CUDA tensor of {k * (ns + 1)} entries")
            ptrs.append(ctypes.c_void_p(arr.data_ptr()))
        self._check(self.L.rtcc_propagate_rk4_mixed(self.ctx, self._state(y), float(t0), float(t_end), float(h1),
                                                    float(h2), ctypes.byref(f), ptrs[0], ptrs[1]))
        return ns

    def step_tableau(self, y, t, h, tab, field=None, tol=1e-10, max_iter=100):
        """One step of any tableau (Tableau or a built-in name); y advances in place. Returns (delta, sweeps):
        the embedded error estimate of an explicit pair (None otherwise) and the implicit stage sweeps (1 for
        explicit tableaux)."""
        T = Tableau.builtin(tab) if isinstance(tab, (str, int)) else tab
        f = field if field is not None else Field.none()
        dl, sw = ctypes.c_double(float("nan")), ctypes.c_int(0)
        self._check(self.L.rtcc_step_tableau(self.ctx, self._state(y), float(t), float(h), ctypes.byref(T),
                                             ctypes.byref(f), float(tol), int(max_iter), ctypes.byref(dl),
                                             ctypes.byref(sw)))
        return (dl.value if T.err_order > 0 else None), sw.value

    def propagate_embedded(self, y, t0, t_end, h0, eps, tab, field=None, record=True, cap=1 << 20,
                           max_trials=1 << 24):
        """Adaptive propagation with an embedded explicit tableau (Tableau or "cashkarp" / "rkf45"); the
        returns of propagate_cashkarp."""
        T = Tableau.builtin(tab) if isinstance(tab, (str, int)) else tab
        return self._adaptive(self.L.rtcc_propagate_embedded, (ctypes.byref(T),), y, t0, t_end, h0, eps, field,
                              record, cap, max_trials)

    def propagate_cashkarp(self, y, t0, t_end, h0, eps, field=None, record=True, cap=1 << 20, max_trials=1 << 24):
        """Adaptive Cash-Karp from t0 to t_end. Returns (times, dipoles (k, 3) complex, n_accepted, n_rejected,
        h_next); times/dipoles are those after every accepted step (empty without record)."""
        return self._adaptive(self.L.rtcc_propagate_cashkarp, (), y, t0, t_end, h0, eps, field, record, cap,
                              max_trials)

    def _adaptive(self, fn, extra, y, t0, t_end, h0, eps, field, record, cap, max_trials):
        f = field if field is not None else Field.none()
        na, nr, hn = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
        if record:
            tt = np.zeros(cap)
            mm = np.zeros(6 * cap)
            tp, mp = _dptr(tt), _dptr(mm)
        else:
            tt = mm = None
            tp = mp = None
        self._check(fn(self.ctx, self._state(y), float(t0), float(t_end), float(h0), float(eps), *extra,
                       ctypes.byref(f), int(max_trials), int(cap) if record else 0, tp, mp, ctypes.byref(na),
                       ctypes.byref(nr), ctypes.byref(hn)))
        k = na.value
        if record:
            m = mm[:6 * k].reshape(k, 6)
            return tt[:k].copy(), m[:, 0::2] + 1j * m[:, 1::2], k, nr.value, hn.value
        return np.zeros(0), np.zeros((0, 3), complex), k, nr.value, hn.value

    def rhs_vjp(self, y, E, ybar, out=None, t=0.0, want_E=False):
        """J^H ybar at (y, E); with want_E also the gradient with respect to the field vector E."""
        if out is None:
            out = self.new_state()
        Ea = (ctypes.c_double * 3)(*[float(x) for x in E])
        Eb = np.zeros(3) if want_E else None
        self._check(self.L.rtcc_rhs_vjp(self.ctx, self._state(y), float(t), Ea, self._state(ybar, "ybar"),
                                        self._state(out, "out"), _dptr(Eb) if want_E else None))
        return (out, Eb) if want_E else out

    def dipole_vjp(self, y, mubar, ybar):
        """ybar += gradient of Re sum_a conj(mubar_a) mu_a(y); mubar: 3 complex numbers."""
        mb = np.asarray(mubar, dtype=np.complex128).reshape(3)
        arr = np.ascontiguousarray(np.stack([mb.real, mb.imag], axis=1).reshape(6))
        self._check(self.L.rtcc_dipole_vjp(self.ctx, self._state(y), _dptr(arr), self._state(ybar, "ybar")))

    def step_rk4_vjp(self, y, t, h, field, ybar, pbar=None):
        """Adjoint of step_rk4 from (y, t): ybar in/out; returns pbar (+= pulse-parameter gradient)."""
        f = field if field is not None else Field.none()
        pb = np.zeros(4) if pbar is None else pbar
        self._check(self.L.rtcc_step_rk4_vjp(self.ctx, self._state(y), float(t), float(h), ctypes.byref(f),
                                             self._state(ybar, "ybar"), _dptr(pb)))
        return pb

    def dipole(self, y):
        out = np.zeros(6)
        self._check(self.L.rtcc_dipole(self.ctx, self._state(y), _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def dipole_dev(self, y, out6):
        self._check(self.L.rtcc_dipole_dev(self.ctx, self._state(y), ctypes.c_void_p(out6.data_ptr())))

    def ground_state(self, y, tol=1e-12, maxiter=200):
        e = ctypes.c_double(0.0)
        self._check(self.L.rtcc_ground_state(self.ctx, self._state(y), float(tol), int(maxiter), ctypes.byref(e)))
        return e.value

    def kick(self, y, kappa, n):
        na = (ctypes.c_double * 3)(*[float(x) for x in n])
        self._check(self.L.rtcc_kick(self.ctx, self._state(y), float(kappa), na))

    def check_state(self, y):
        k = ctypes.c_int64(0)
        self._check(self.L.rtcc_check_state(self.ctx, self._state(y), ctypes.byref(k)))
        return k.value

    def profile(self, enable=True, target="ladder"):
        """Time the ladder GEMMs (target "ladder") or the large complex x complex products ("complex")."""
        mode = {"ladder": 1, "complex": 2}[target] if enable else 0
        self._check(self.L.rtcc_profile(self.ctx, mode))

    def profile_read(self):
        """(timed launches, summed ms, algorithmic flops per launch, algorithmic bytes per launch)."""
        n, ms, fl, by = ctypes.c_int64(0), ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(self.L.rtcc_profile_read(self.ctx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                             ctypes.byref(by)))
        return n.value, ms.value, fl.value, by.value

    def info(self):
        out = (ctypes.c_int64 * 6)()
        self._check(self.L.rtcc_info(self.ctx, out))
        return {"o": out[0], "v": out[1], "nstate": out[2], "last_rhs_flops": out[3],
                "device_bytes": out[4], "precision": out[5]}

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.L.rtcc_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_batch(systems, ys, fields, t0, h, nsteps, mu_out=None):
    """Batched RK4 propagation (rtcc_propagate_batch).

    systems: list of RTCC contexts (distinct); ys[s]: contiguous complex128 CUDA tensor of shape
    (members_s, state_size); fields[s]: list of members_s Field; mu_out: None or a list with, per
    system, None or a contiguous float64 CUDA tensor of (nsteps+1) * members_s * 6 entries.
    Ordered on the stream of systems[0].
    """
    import torch
    nsys = len(systems)
    if nsys == 0 or len(ys) != nsys or len(fields) != nsys:
        raise ValueError("systems, ys and fields must have one entry per system")
    L = systems[0].L
    nprop = []
    for R, y, fl in zip(systems, ys, fields):
        if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.complex128 and y.is_contiguous()
                and y.dim() == 2 and y.shape[1] == R.nstate and y.shape[0] == len(fl) and y.shape[0] > 0):
            raise ValueError("ys[s] must be a contiguous complex128 CUDA tensor (members, state_size) "
                             "matching fields[s]")
        nprop.append(y.shape[0])
    flat = [f for fl in fields for f in fl]
    ctxs = (ctypes.c_void_p * nsys)(*[R.ctx.value for R in systems])
    npa = (ctypes.c_int * nsys)(*nprop)
    ypa = (ctypes.c_void_p * nsys)(*[y.data_ptr() for y in ys])
    fa = (Field * len(flat))(*flat)
    mpa = None
    if mu_out is not None:
        ptrs = []
        for m, k in zip(mu_out, nprop):
            if m is None:
                ptrs.append(None)
                continue
            if not (m.is_cuda and m.dtype == torch.float64 and m.is_contiguous() and m.numel() >= 6 * k * (nsteps + 1)):
                raise ValueError("mu_out[s] must be a contiguous float64 CUDA tensor of (nsteps+1)*members*6 entries")
            ptrs.append(m.data_ptr())
        mpa = (ctypes.c_void_p * nsys)(*ptrs)
    rc = L.rtcc_propagate_batch(ctxs, nsys, npa, ypa, fa, float(t0), float(h), int(nsteps), mpa)
    systems[0]._check(rc)


def mixed_schedule(t0, t_end, h1, h2, field=None):
    """Times (t0 and every step end) of the mixed step-size RK4 schedule (rtcc_mixed_schedule)."""
    L = load_library()
    f = field if field is not None else Field.none()
    n = ctypes.c_int(0)
    rc = L.rtcc_mixed_schedule(float(t0), float(t_end), float(h1), float(h2), ctypes.byref(f), 0, None,
                               ctypes.byref(n))
    if rc != 0:
        raise RTCCError(rc, L.rtcc_last_error(None).decode())
    times = np.zeros(n.value + 1)
    rc = L.rtcc_mixed_schedule(float(t0), float(t_end), float(h1), float(h2), ctypes.byref(f), times.size,
                               _dptr(times), ctypes.byref(n))
    if rc != 0:
        raise RTCCError(rc, L.rtcc_last_error(None).decode())
    return times


def check_state_noalloc(o, v, y, out, stream=None):
    """rtcc_check_state_noalloc: out (float64 CUDA tensor, 2 entries) = (|T2|, non-finite count) of the
    state y, enqueued on the stream without any allocation or synchronisation."""
    import torch
    L = load_library()
    st = stream if stream is not None else torch.cuda.current_stream()
    if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 2 and y.is_cuda and
            y.dtype == torch.complex128 and y.numel() == state_size(o, v)):
        raise ValueError("y must be a complex128 CUDA state of (o, v) and out a float64 CUDA tensor of 2 entries")
    rc = L.rtcc_check_state_noalloc(int(o), int(v), ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RTCCError(rc, L.rtcc_last_error(None).decode())


def peak_probe(kind, size):
    """rtcc_peak_probe: "fp64" / "fp32" / "bf16" MFMA rate in TFLOP/s (size = rounds per wave) or "copy"
    HBM copy bandwidth in GB/s (size = bytes per buffer), measured on the current device."""
    L = load_library()
    k = {"fp64": 0, "fp32": 1, "bf16": 2, "copy": 3}[kind]
    v = ctypes.c_double(0.0)
    rc = L.rtcc_peak_probe(k, int(size), ctypes.byref(v))
    if rc != 0:
        raise RTCCError(rc, L.rtcc_last_error(None).decode())
    return v.value


def state_size(o, v):
    return 2 * (o * v + (o * v) ** 2)
