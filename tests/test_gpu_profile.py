"""Live kernel timing (rtcc_profile / rtcc_profile_read) times exactly the launches it is meant to time.

Mode 2 ("complex") brackets every complex x complex product with 2 M N K >= 5e8 -- in the
split-BF16 context only launches of the register-staged 128 x 256 kernel, where a launch may carry the
two or three independent products of a Lambda1 group -- and mode 1 ("ladder") the
ladder GEMMs. One right-hand side at (16,42) (complex products of 672 x 672 and 256 x 672 outputs, the
split-BF16 ones on 18-tile grids, so the 128 x 256 kernel runs) is evaluated with the engine trace on;
the trace's GEMM lines give the expected launch count and flop sum (8 M N K per complex product), which
profile_read must reproduce, with a positive elapsed time and at least the operand-and-output bytes per
launch, also over RK4 steps that fill the event buffer mid-step; the ladder mode times its two GEMMs (two launches here: neither reaches the split-BF16 threshold,
so they are not paired) with their flops. An unknown mode is refused.
"""
import re

import numpy as np
import pytest

from synth import make_system, pack_state, random_state

pytestmark = pytest.mark.gpu

O, V = 16, 42


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _expected(trace, prec):
    """(launches, summed flops, summed minimum bytes, grouped launches) of the complex products the trace
    shows."""
    n, fl, by, ng = 0, 0.0, 0.0, 0
    esz = 16 if prec == "fp64" else 8
    for line in trace.splitlines():
        if prec == "bf16x3":
            # single products, and the products issued together as one launch ("multi h/n")
            g = re.search(r"\[rtcc\] gemm-bf16x3 multi (\d)/\d M=(\d+) N=(\d+) K=(\d+) cc ", line)
            if g:
                M, N, K = int(g[2]), int(g[3]), int(g[4])
                n += g[1] == "1"
                ng += g[1] == "1"
                fl += 8.0 * M * N * K
                by += esz * (M * K + K * N + M * N)
                continue
            m = re.search(r"\[rtcc\] gemm-bf16x3 M=(\d+) N=(\d+) K=(\d+) cc .* wn=(\d) splits=\d+ kernel=(\d)", line)
            if not m or m[4] != "4" or m[5] != "1":
                continue
            M, N, K, nb = int(m[1]), int(m[2]), int(m[3]), 1
        else:
            m = re.search(r"\[rtcc\] gemm M=(\d+) N=(\d+) K=(\d+) batch=(\d+) cc ", line)
            if not m:
                continue
            M, N, K, nb = (int(x) for x in m.groups())
            if 2.0 * M * N * K * nb < 5e8:
                continue
        n += 1
        fl += 8.0 * M * N * K * nb
        by += esz * nb * (M * K + K * N + M * N)
    return n, fl, by, ng


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_complex_product_timing_counts_the_traced_products(monkeypatch, capfd, prec):
    import torch
    from paper_2205_05175_amd import RTCC, RTCCError
    print(f"profile mode 2 at ({O},{V}) {prec}", flush=True)
    monkeypatch.setenv("RTCC_TRACE", "1")
    R = RTCC(*make_system(O, V, 0), O, V, prec)
    y = torch.tensor(pack_state(*random_state(O, V, 5, 0.02, 0.01)), device="cuda")
    R.rhs(y, [0.0, 0.0, 0.001])  # first call: constant operands packed and cached
    torch.cuda.synchronize()
    capfd.readouterr()
    R.profile(True, "complex")
    R.rhs(y, [0.0, 0.0, 0.001])
    n, ms, fl, by = R.profile_read()
    R.profile(False)
    trace = capfd.readouterr().err
    en, efl, eby, eng = _expected(trace, prec)
    print(f"  timed {n} launches, {ms:.3f} ms, {fl:.4g} flop and {by:.4g} B per launch; trace {en} "
          f"({eng} grouped)", flush=True)
    # ten complex products with 2 M N K >= 5e8; in the split-BF16 context the two Lambda1 groups of three
    # independent products go out as one launch each
    assert n == en and en == (6 if prec == "bf16x3" else 10) and eng == (2 if prec == "bf16x3" else 0)
    assert fl * n == pytest.approx(efl, rel=1e-12)
    assert ms > 0.0
    # the bytes count the output once more where a product accumulates into it
    assert eby <= by * n <= eby * 2
    # RK4 steps issued eagerly while profiling, enough of them to fill the event buffer (512 pairs)
    # mid-step: every launch is still timed
    y2 = y.clone()
    R.profile(True, "complex")
    R.propagate_rk4(y2, 0.0, 0.01, 15)
    n2, ms2, fl2, _ = R.profile_read()
    R.profile(False)
    assert n2 == 15 * 4 * en and fl2 == pytest.approx(fl, rel=1e-12) and ms2 > ms
    # the ladder: its two GEMMs, in one launch when both take the split-BF16 kernel (2 M N K >= 5e8:
    # not at this size, where the rows are o(o+1) = 272 and o(o-1) = 240 for tau and lambda2)
    rows = (O * (O + 1), O * (O - 1))
    kn = (V * (V + 1) // 2, V * (V - 1) // 2)
    paired = prec == "bf16x3" and all(2.0 * r * k * k >= 5e8 for r, k in zip(rows, kn))
    R.profile(True, "ladder")
    R.rhs(y, [0.0, 0.0, 0.001])
    nl, msl, fll, byl = R.profile_read()
    R.profile(False)
    assert nl == (1 if paired else 2) and msl > 0.0 and byl == 0.0
    assert fll * nl == pytest.approx(4.0 * O * (O + 1) * (V * (V + 1) // 2) ** 2
                                     + 4.0 * O * (O - 1) * (V * (V - 1) // 2) ** 2, rel=1e-12)
    with pytest.raises(RTCCError):
        R._check(R.L.rtcc_profile(R.ctx, 3))
    R.close()
