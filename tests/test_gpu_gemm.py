"""Every GEMM kernel the autotuner may pick, through rtcc_gemm, against an FP64 host product.

The shapes cover the production kernels and their edge cases at sizes the host checks in seconds:
the ladder form (complex rows x real symmetric matrix), a complex x complex ring product with more
than eight 128-row tile rows (the multi-band XCD numbering of the split-BF16 kernel), transposed
operands of both kinds, ragged extents (not multiples of any tile), skinny outputs with long K, and
accumulation into C (beta = 1). Tolerances are relative to the largest entry of the exact product:
FP64 1e-12, FP32 2e-5 (single rounding over K terms), split-BF16 1e-4 (hi + lo represent each operand
to ~2^-17 relative). Finally the tuning table: a listed shape runs the listed kernel (bitwise the same
result as forcing it, and a different rounding from the library's own rule).
"""
import ctypes
import os
import tempfile

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 1e-4}
TAG = {"fp64": 0, "fp32": 1, "bf16x3": 2}
TILES = [(64064, 16), (128128, 16), (32064, 32), (32128, 16), (64032, 32), (64096, 32), (32032, 64), (32096, 32),
         (96032, 32), (32096, 64), (64032, 64), (32064, 64)]


class Case:
    def __init__(self, M, N, K, ac, bc, ta, tb, seed=0):
        rng = np.random.default_rng(seed)
        mk = lambda r, c: rng.normal(0.0, 0.1, size=(r, c))
        self.shape = (M, N, K, ac, bc, ta, tb)
        a = mk(M, K) + (1j * mk(M, K) if ac else 0)
        b = mk(K, N) + (1j * mk(K, N) if bc else 0)
        self.a, self.b = a, b
        self.c0 = mk(M, N) + (1j * mk(M, N) if (ac or bc) else 0)

    def ref(self, alpha, beta):
        return alpha * (self.a @ self.b) + beta * self.c0


def _run(prec, case, choice, alpha=1.0, beta=0.0):
    import torch
    from paper_2205_05175_amd import load_library
    L = load_library()
    M, N, K, ac, bc, ta, tb = case.shape
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    A = case.a.T if ta else case.a
    B = case.b.T if tb else case.b
    ar, ai = dev(A.real), (dev(A.imag) if ac else None)
    br, bi = dev(B.real), (dev(B.imag) if bc else None)
    cc = ac or bc
    cr, ci = dev(case.c0.real), (dev(case.c0.imag) if cc else None)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    ch = (ctypes.c_int * 4)(*choice) if choice is not None else None
    rc = L.rtcc_gemm(TAG[prec], M, N, K, alpha, p(ar), p(ai), A.shape[1], ta, p(br), p(bi), B.shape[1], tb, beta,
                     p(cr), p(ci), N, ch, 0, None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        return None
    out = cr.cpu().numpy().astype(np.float64)
    if cc:
        out = out + 1j * ci.cpu().numpy()
    return out


def _check(prec, case, choice, alpha=1.0, beta=0.0, must_run=True):
    got = _run(prec, case, choice, alpha, beta)
    if got is None:
        assert not must_run, f"{prec} {case.shape} choice {choice} was refused"
        return None
    ref = case.ref(alpha, beta)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < TOL[prec], f"{prec} {case.shape} choice {choice}: rel error {err:.3e}"
    return err


SHAPES = [
    (200, 1444, 1444, True, False, False, True),   # ladder form: [tau; lambda2] x <ef|ab>^T
    (1100, 1100, 2200, True, True, False, True),   # ring form, 9 tile rows of 128
    (300, 257, 515, False, True, True, False),     # transposed real A, ragged
    (129, 333, 700, True, True, True, True),       # both transposed, ragged
    (20, 1520, 76, True, False, False, False),     # short K, thin M
    (20, 76, 11552, True, True, False, True),      # small output, long K
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(str(int(x)) for x in s))
def test_every_kernel_choice_matches_host(shape):
    case = Case(*shape)
    M, N, K, ac, bc, ta, tb = shape
    print(f"gemm kernels {shape}", flush=True)
    for prec in ("fp64", "fp32", "bf16x3"):
        _check(prec, case, None)
        for mn, bk in TILES:
            if mn == 128128 and prec == "fp64":
                continue
            for s in (1, 3, 8):
                if s > 1 and K // s < bk:
                    continue
                # thin tiles need 16-byte aligned operands: refused otherwise, never wrong
                _check(prec, case, (1, mn, bk, s), must_run=mn in (64064, 128128))
        if prec == "bf16x3":
            # register-staged, direct-to-LDS ring, the ring at two per CU, wide waves
            for kern, wns in ((1, (2, 4)), (2, (2, 4)), (3, (2,)), (4, (4,))):
                for wn in wns:
                    for s in (1, 2, 5):
                        _check(prec, case, (2, wn, kern, s))
    # accumulation into C
    _check("fp32", case, (1, 64064, 16, 1), alpha=0.5, beta=1.0)
    _check("bf16x3", case, (2, 4, 1, 1), alpha=0.5, beta=1.0)
    _check("bf16x3", case, (2, 2, 2, 3), alpha=-1.0, beta=1.0)
    _check("bf16x3", case, (2, 4, 2, 1), alpha=0.5, beta=1.0)
    _check("bf16x3", case, (2, 2, 3, 2), alpha=0.5, beta=1.0)
    _check("bf16x3", case, (2, 4, 4, 1), alpha=-0.5, beta=1.0)
    _check("fp64", case, (1, 64064, 16, 4), alpha=2.0, beta=1.0)


def test_tuning_table_is_used():
    from paper_2205_05175_amd import TUNING_PATH, load_library
    L = load_library()
    case = Case(300, 260, 4100, True, True, False, True)
    base = _run("fp32", case, (1, 64064, 16, 1))
    forced = _run("fp32", case, (1, 64064, 16, 8))
    assert base is not None and forced is not None
    assert not np.array_equal(base, forced)  # eight partial sums round differently
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as fh:
        fh.write("# test table\n1 300 260 4100 1 1 0 1 1 64064 16 8\n")
        path = fh.name
    try:
        n = ctypes.c_int(0)
        assert L.rtcc_load_tuning(path.encode(), ctypes.byref(n)) == 0 and n.value == 1
        tuned = _run("fp32", case, None)
        assert np.array_equal(tuned, forced)
        with open(path, "w") as fh:
            fh.write("1 300 260 4100 1 1 0 one 1 64064 16 8\n")
        assert L.rtcc_load_tuning(path.encode(), None) == -1  # malformed: rejected, table unchanged
        assert np.array_equal(_run("fp32", case, None), forced)
    finally:
        os.unlink(path)
        L.rtcc_load_tuning(TUNING_PATH.encode() if os.path.exists(TUNING_PATH) else None, None)
