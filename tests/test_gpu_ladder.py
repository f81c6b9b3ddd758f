"""The symmetric / antisymmetric particle-particle ladder (the default) against the full product.

The right-hand side with the two triangle GEMMs (X+ V+ over i <= j, e <= f and X- V- over i < j, e < f)
must equal the right-hand side with the single o^2 v^2 x v^2 ladder GEMM (RTCC_LADDER=full) to rounding,
and the oracle (which sums the ladder over all e, f) in every precision. Sizes: o = 1 (no antisymmetric
rows), v = 1 (no antisymmetric columns), ragged triangles that span several tiles ((7,36): 28 x 666 and
21 x 630 per block), and the batched path (member-contiguous triangles).
"""
import numpy as np
import pytest

from oracle import ccsd
from synth import make_system, pack_state, random_state, random_symmetric, unpack_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _case(o, v, seed=3):
    eri, fock, mu = make_system(o, v, seed)
    fock = fock + random_symmetric(o + v, 0.05, np.random.default_rng(1000 + seed))
    return eri, fock, mu, pack_state(*random_state(o, v, 40 + seed, 0.05, 0.02))


def _rhs(monkeypatch, mode, eri, fock, mu, o, v, y, prec, E):
    import torch
    from paper_2205_05175_amd import RTCC
    monkeypatch.setenv("RTCC_LADDER", mode)
    R = RTCC(eri, fock, mu, o, v, prec)
    out = R.rhs(torch.tensor(y, device="cuda"), E)
    got = out.cpu().numpy()
    R.close()
    return got


@pytest.mark.parametrize("o,v", [(1, 5), (3, 1), (2, 3), (4, 16), (7, 36)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("bf16x3", 3e-4)])
def test_symmetric_ladder_equals_full_and_oracle(monkeypatch, o, v, prec, tol):
    print(f"symmetric ladder o={o} v={v} {prec}", flush=True)
    monkeypatch.setenv("RTCC_BF16_MIN_FLOPS", "0")
    eri, fock, mu, y = _case(o, v)
    E = [0.003, -0.002, 0.01]
    sym = _rhs(monkeypatch, "symmetric", eri, fock, mu, o, v, y, prec, E)
    full = _rhs(monkeypatch, "full", eri, fock, mu, o, v, y, prec, E)
    # the element fold / unfold kernels (used beyond v = 96) give the same numbers as the LDS-staged ones
    nolds = _rhs(monkeypatch, "symmetric-nolds", eri, fock, mu, o, v, y, prec, E)
    assert np.array_equal(sym, nolds)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    ref = pack_state(*ccsd.rhs(S, *unpack_state(y, o, v), np.array(E)))
    scale = np.abs(ref).max()
    assert np.abs(sym - ref).max() < tol * scale
    assert np.abs(full - ref).max() < tol * scale
    if prec == "fp64":
        assert np.abs(sym - full).max() < 1e-12 * scale


def test_symmetric_ladder_in_batched_step(monkeypatch):
    """Batched RK4 steps (members of two sizes) with the symmetric ladder equal the same steps with the
    full ladder (FP64, eager launches: the captured FP64 batch has a skipped case of its own)."""
    import torch
    from paper_2205_05175_amd import RTCC, Field, propagate_batch
    print("symmetric ladder in a batched step (3,8) x 3 + (2,5) x 2 fp64", flush=True)
    outs = {}
    monkeypatch.setenv("RTCC_NO_GRAPH", "1")
    for mode in ("symmetric", "full"):
        monkeypatch.setenv("RTCC_LADDER", mode)
        systems, ys, fields = [], [], []
        for (o, v), nm in (((3, 8), 3), ((2, 5), 2)):
            eri, fock, mu, _ = _case(o, v, seed=o)
            R = RTCC(eri, fock, mu, o, v, "fp64")
            systems.append(R)
            ys.append(torch.stack([torch.tensor(pack_state(*random_state(o, v, 60 + k, 0.05, 0.02)), device="cuda")
                                   for k in range(nm)]))
            fields.append([Field.gaussian(0.01 * (k + 1), 0.5, 1.0, 0.5, [0.0, 0.0, 1.0]) for k in range(nm)])
        propagate_batch(systems, ys, fields, 0.0, 0.05, 3, None)
        torch.cuda.synchronize()
        outs[mode] = [y.cpu().numpy() for y in ys]
        for R in systems:
            R.close()
    for a, b in zip(outs["symmetric"], outs["full"]):
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
