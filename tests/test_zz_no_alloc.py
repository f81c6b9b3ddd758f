"""rtcc_check_state_noalloc (the allocation-free entry point) against rtcc_check_state.

Two calls in a row on one GPU, the second with a smaller state: the non-finite counts must equal
rtcc_check_state's exactly, and |T2| must equal the Frobenius norm of the T2 block computed on the
host (FP64 sums in a different order: 1e-13 relative), or be NaN when the state has a non-finite entry.
"""
import ctypes

import numpy as np
import pytest

from synth import make_system, pack_state, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _noalloc(L, o, v, y, out):
    import torch
    rc = L.rtcc_check_state_noalloc(o, v, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.rtcc_last_error(None)
    torch.cuda.synchronize()
    return out.cpu().numpy().copy()


def test_noalloc_check_matches_check_state():
    import torch
    from paper_2205_05175_amd import RTCC
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    cases = [(5, 19, []), (2, 3, [1, 17, 40])]  # second call: smaller state, three NaN / Inf entries
    for o, v, bad in cases:
        print(f"no-alloc check o={o} v={v} bad={bad}", flush=True)
        R = RTCC(*make_system(o, v, 0), o, v, "fp64")
        st = random_state(o, v, 4, 0.05, 0.02)
        yh = pack_state(*st)
        for k, i in enumerate(bad):
            yh[i] = [np.nan, np.inf + 0j, complex(0.0, -np.inf)][k % 3]
        y = torch.tensor(yh, device="cuda")
        got = _noalloc(R.L, o, v, y, out)
        assert got[1] == R.check_state(y) == len(bad)
        if bad:
            assert np.isnan(got[0])
        else:
            ref = np.linalg.norm(st[1])
            assert abs(got[0] - ref) < 1e-13 * ref
        R.close()
    # invalid sizes are rejected without launching anything
    from paper_2205_05175_amd import load_library
    L = load_library()
    assert L.rtcc_check_state_noalloc(0, 5, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    assert L.rtcc_check_state_noalloc(1 << 11, 1 << 11, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
