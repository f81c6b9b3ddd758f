"""Write sampled oracle right-hand-side values at the production size (o, v) = (20, 76).

Calls only the oracle (``oracle/``) and the seeded input generator (``synth``). One right-hand side of
the spin-orbital oracle at this size needs ~11 GB for the antisymmetrised integrals and ~50 GB at its
peak, and minutes of host time, so it is evaluated once here and a seeded sample of its entries is
stored; the GPU test compares the library's right-hand side (FP64, FP32 and split-BF16, in the launch
configuration of the benchmark) with these entries.

Case: synth.make_system(20, 76, seed=0), a random non-stationary state synth.random_state(20, 76, 3,
0.05, 0.02), field E = (0.003, -0.002, 0.01) au. Samples: 4096 indices of the packed state drawn
with numpy.random.default_rng(20) (uniform over the whole state, so each of T1, T2, L1, L2 in
proportion to its size), plus all of T1 and L1 (1520 entries each), which the doubles would outnumber.

Usage: python tests/golden/make_fullsize.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ccsd  # noqa: E402
from synth import make_system, pack_state, random_state, state_size  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
O, V, SEED, STATE_SEED = 20, 76, 0, 3
E = [0.003, -0.002, 0.01]


def main():
    t0 = time.time()
    eri, fock, mu = make_system(O, V, SEED)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, O, V)
    del eri
    print(f"spin-orbital integrals built in {time.time() - t0:.0f} s", flush=True)
    st = random_state(O, V, STATE_SEED, 0.05, 0.02)
    t1 = time.time()
    d = pack_state(*ccsd.rhs(S, *st, np.array(E)))
    t_rhs = time.time() - t1
    print(f"one oracle RHS in {t_rhs:.0f} s", flush=True)
    n = state_size(O, V)
    n1, n2 = O * V, (O * V) ** 2
    rng = np.random.default_rng(20)
    idx = set(rng.integers(0, n, size=4096).tolist())
    idx.update(range(n1))                      # T1
    idx.update(range(n1 + n2, 2 * n1 + n2))    # L1
    idx = np.array(sorted(idx))
    out = dict(case=dict(o=O, v=V, seed=SEED, state_seed=STATE_SEED, scale1=0.05, scale2=0.02, E=E),
               index=idx.tolist(), value=[[float(z.real), float(z.imag)] for z in d[idx]],
               max_abs_all=float(np.abs(d).max()), oracle_rhs_seconds=t_rhs,
               generator="tests/golden/make_fullsize.py (oracle, spin-orbital FP64)")
    with open(os.path.join(HERE, "rhs_o20v76_samples.json"), "w") as fh:
        json.dump(out, fh)
    print(f"wrote {idx.size} samples", flush=True)


if __name__ == "__main__":
    main()
