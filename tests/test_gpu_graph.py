"""The captured RK4 step (one hipGraph replayed every step) equals the eager launch sequence bitwise.

In FP32 and split-BF16 contexts the captured step computes the dipole of its start state on a fourth
stream beside the right-hand sides (and the final state's dipole after the last step); the eager
sequence computes each step's end-state dipole after the step: the recorded dipoles must agree bitwise."""
import os

import numpy as np
import pytest

from synth import make_system, pack_state, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


def _ctx(o, v, precision, graph):
    from paper_2205_05175_amd import RTCC
    eri, fock, mu = make_system(o, v, 3)
    old = os.environ.get("RTCC_NO_GRAPH")
    os.environ["RTCC_NO_GRAPH"] = "0" if graph else "1"
    try:
        return RTCC(eri, fock, mu, o, v, precision)
    finally:
        if old is None:
            del os.environ["RTCC_NO_GRAPH"]
        else:
            os.environ["RTCC_NO_GRAPH"] = old


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_graph_replays_match_eager(precision):
    import torch
    from paper_2205_05175_amd import Field
    o, v = 4, 16
    fld = Field.gaussian(0.02, 0.5, 1.0, 0.3, [0.2, 0.3, 0.9])
    y0 = torch.tensor(pack_state(*random_state(o, v, 5, 0.05, 0.02)), device="cuda")
    Rg, Re = _ctx(o, v, precision, True), _ctx(o, v, precision, False)
    yg, ye = y0.clone(), y0.clone()
    h, t = 0.05, 0.0
    for k in range(6):
        mg = torch.zeros((2, 6), dtype=torch.float64, device="cuda")
        me = torch.zeros((2, 6), dtype=torch.float64, device="cuda")
        Rg.propagate_rk4(yg, t, h, 1, fld, mg)   # replay of the same captured step (after the first)
        Re.propagate_rk4(ye, t, h, 1, fld, me)
        # eager work and a synchronisation between replays
        dg = Rg.dipole(yg)
        torch.cuda.synchronize()
        assert torch.equal(yg, ye), f"state differs after step {k}"
        assert torch.equal(mg, me)
        assert np.array_equal(dg, Re.dipole(ye))
        t += h
    # a multi-step call replays the graph nsteps times
    mg = torch.zeros((5, 6), dtype=torch.float64, device="cuda")
    me = torch.zeros((5, 6), dtype=torch.float64, device="cuda")
    Rg.propagate_rk4(yg, t, h, 4, fld, mg)
    Re.propagate_rk4(ye, t, h, 4, fld, me)
    torch.cuda.synchronize()
    assert torch.equal(yg, ye) and torch.equal(mg, me)
