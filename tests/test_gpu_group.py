"""Grouped launches of independent products (ein_multi / gemm_bf16x3_multi) in the split-BF16 context.

One right-hand side at (16,42), where the two Lambda1 groups of three l2s x t2 products (672 x 672 x 672,
complex x complex) and the two ring-formation products (real x complex) go out grouped:
* grouped = one launch per product (RTCC_NO_GROUP=1) up to the rounding of their different K splits;
* with tuning-table entries for the grouped shapes every group falls back to one launch per product, each
  through the table: bitwise the right-hand side of RTCC_NO_GROUP=1 under the same table;
* the group is really formed (trace lines), and the fallback really happens (no "multi" lines);
* the band height of the workgroup -> output-tile map (RTCC_TILE_BAND) only moves tiles between
  workgroups: any band gives the bitwise right-hand side of the default one.
"""
import ctypes
import os
import re
import tempfile

import numpy as np
import pytest

from synth import make_system, pack_state, random_state

pytestmark = pytest.mark.gpu

O, V = 16, 42


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _rhs(monkeypatch, capfd, group, band="8"):
    import torch
    from paper_2205_05175_amd import RTCC
    monkeypatch.setenv("RTCC_NO_GROUP", "0" if group else "1")
    monkeypatch.setenv("RTCC_TILE_BAND", band)
    monkeypatch.setenv("RTCC_TRACE", "1")
    R = RTCC(*make_system(O, V, 0), O, V, "bf16x3")
    y = torch.tensor(pack_state(*random_state(O, V, 5, 0.02, 0.01)), device="cuda")
    capfd.readouterr()
    out = R.rhs(y, [0.0, 0.0, 0.001]).cpu().numpy()
    trace = capfd.readouterr().err
    R.close()
    return out, trace


def test_grouped_products_match_single_launches(monkeypatch, capfd):
    from paper_2205_05175_amd import TUNING_PATH, load_library
    print(f"grouped launches at ({O},{V}) bf16x3", flush=True)
    g, tg = _rhs(monkeypatch, capfd, True)
    s, ts = _rhs(monkeypatch, capfd, False)
    multi = re.findall(r"\[rtcc\] gemm-bf16x3 multi (\d)/(\d) M=(\d+) N=(\d+) K=(\d+) (\w\w) ta=(\d) tb=(\d)", tg)
    assert sum(1 for m in multi if m[0] == "1") >= 2 and not re.search(r"gemm-bf16x3 multi", ts)
    scale = np.abs(s).max()
    err = np.abs(g - s).max() / scale
    print(f"  {len(multi)} grouped products; grouped vs single launches {err:.2e} (rel.)", flush=True)
    assert err < 3e-5

    # table entries for every grouped shape: each group then goes one product at a time through the table,
    # exactly as without grouping
    shapes = sorted({(int(m[2]), int(m[3]), int(m[4]), int(m[5][0] == "c"), int(m[5][1] == "c"), int(m[6]),
                      int(m[7])) for m in multi})
    L = load_library()
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as fh:
        fh.write("# test table\n")
        for M, N, K, ac, bc, ta, tb in shapes:
            fh.write(f"2 {M} {N} {K} {ac} {bc} {ta} {tb} 2 4 1 3\n")
        path = fh.name
    try:
        n = ctypes.c_int(0)
        assert L.rtcc_load_tuning(path.encode(), ctypes.byref(n)) == 0 and n.value == len(shapes)
        gf, tgf = _rhs(monkeypatch, capfd, True)
        sf, _ = _rhs(monkeypatch, capfd, False)
        print(f"  with table entries for {len(shapes)} shapes: "
              f"{len(re.findall(r'gemm-bf16x3 multi', tgf))} grouped products left", flush=True)
        assert not re.search(r"gemm-bf16x3 multi", tgf)
        assert np.array_equal(gf, sf)
    finally:
        os.unlink(path)
        L.rtcc_load_tuning(TUNING_PATH.encode() if os.path.exists(TUNING_PATH) else None, None)


@pytest.mark.parametrize("band", ["1", "3", "64"])
def test_tile_band_moves_tiles_only(monkeypatch, capfd, band):
    print(f"tile band {band} at ({O},{V}) bf16x3", flush=True)
    ref, _ = _rhs(monkeypatch, capfd, True)
    out, _ = _rhs(monkeypatch, capfd, True, band)
    assert np.array_equal(out, ref)
