"""Tile autotuner for the contraction GEMMs (run it on the GPU it tunes for).

Every term of the right-hand side is a GEMM of a fixed shape for a given system size. This tool
collects the shapes of one right-hand side per contraction precision (from the library's trace of a
call at the requested (o, v)), times every candidate kernel for each shape with ``rtcc_gemm`` on
random operands of that shape and layout, and writes the fastest choice per shape, with the measured
times of the winner and of the library's own rule as comments, into the tuning table that
``rtcc_load_tuning`` reads (the package loads ``tuned_gemm.txt`` beside it at start-up). An entry is
kept only when it beats the library's own rule by more than ``--min-gain``.

Candidates: the tile kernel in each of its tile / k-stage shapes with 1 to 1024 K splits; for
split-BF16 contexts also the split-BF16 kernels (register-staged, direct-to-LDS ring, the ring at two
workgroups per CU) with 128 x 128 or 128 x 256 tiles and 1 to 16 splits, within the workgroup cap the
library applies to split grids.

Usage: python -m paper_2205_05175_amd.autotune --o 20 --v 76 [--out FILE] [--precisions fp64,fp32,bf16x3]
       [--max-flops F]   (only products with 2 M N K < F; the others keep their table entries)
"""
from __future__ import annotations

import argparse
import ctypes
import os
import re
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuned_gemm.txt")
PREC_TAG = {"fp64": 0, "fp32": 1, "bf16x3": 2}
# (bm * 1000 + bn, k stage, aligned operands only) as instantiated by the library's dispatcher
TILES = [(64064, 16, False), (128128, 16, False), (32064, 32, True), (32128, 16, True), (64032, 32, True),
         (64096, 32, True), (32032, 64, True), (32096, 32, True), (96032, 32, True), (32096, 64, True),
         (64032, 64, True), (32064, 64, True)]
SPLITS = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 128, 256, 512, 1024]

_LINE = re.compile(r"\[rtcc\] gemm(-bf16x3)? M=(\d+) N=(\d+) K=(\d+)(?: batch=(\d+))? ([cr])([cr]) ta=(\d) tb=(\d)")

_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2205_05175_amd import RTCC, Field, propagate_batch
from synth import make_system, pack_state, random_state
o, v, prec, nb = int(sys.argv[2]), int(sys.argv[3]), sys.argv[4], int(sys.argv[5])
R = RTCC(*make_system(o, v, 0), o, v, prec)
if nb == 0:
    y = torch.tensor(pack_state(*random_state(o, v, 3)), device="cuda")
    R.rhs(y, [0.001, 0.0, 0.002])
else:
    # one batched RK4 step of nb members (eager launches: every product is traced)
    ys = torch.tensor(np.stack([pack_state(*random_state(o, v, 3 + m)) for m in range(nb)]), device="cuda")
    propagate_batch([R], [ys], [[Field.none() for _ in range(nb)]], 0.0, 0.02, 1, None)
torch.cuda.synchronize()
"""


def collect_shapes(o, v, prec, batch=0):
    """(M, N, K, ac, bc, ta, tb) of the non-batched GEMMs of one right-hand side in precision prec (with
    batch > 0: of one batched RK4 step of that many members, whose member-folded products are single GEMMs)."""
    env = dict(os.environ, RTCC_TRACE="1", RTCC_NO_TUNING="1", RTCC_NO_GRAPH="1")
    root = os.path.dirname(HERE)
    r = subprocess.run([sys.executable, "-c", _CHILD, root, str(o), str(v), prec, str(batch)], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"shape collection failed:\n{r.stderr[-2000:]}")
    shapes = {}
    for line in r.stderr.splitlines():
        m = _LINE.search(line)
        if not m:
            continue
        if m.group(5) is not None and int(m.group(5)) != 1:
            continue
        M, N, K = int(m.group(2)), int(m.group(3)), int(m.group(4))
        if M <= 1 or N <= 1:
            continue
        key = (M, N, K, m.group(6) == "c", m.group(7) == "c", int(m.group(8)), int(m.group(9)))
        shapes[key] = shapes.get(key, 0) + 1
    return shapes


class Operands:
    """Random device operands of one shape (contiguous, leading dimensions of the stored layout)."""

    def __init__(self, M, N, K, ac, bc, ta, tb, prec):
        import torch
        dt = torch.float64 if prec == "fp64" else torch.float32
        g = torch.Generator(device="cuda").manual_seed(1234)
        mk = lambda r, c: torch.randn(r, c, dtype=dt, device="cuda", generator=g) * 0.1
        self.ar = mk(K, M) if ta else mk(M, K)
        self.ai = (mk(K, M) if ta else mk(M, K)) if ac else None
        self.br = mk(N, K) if tb else mk(K, N)
        self.bi = (mk(N, K) if tb else mk(K, N)) if bc else None
        self.cr = torch.zeros(M, N, dtype=dt, device="cuda")
        self.ci = torch.zeros(M, N, dtype=dt, device="cuda") if (ac or bc) else None
        self.lda, self.ldb, self.ldc = (M if ta else K), (K if tb else N), N
        self.shape = (M, N, K, ac, bc, ta, tb)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def run_gemm(L, prec, ops, choice=None, reps=0, alpha=1.0, beta=0.0):
    """rtcc_gemm on the operands; returns the mean time (ms) when reps > 0."""
    import torch
    M, N, K, ac, bc, ta, tb = ops.shape
    ch = (ctypes.c_int * 4)(*choice) if choice is not None else None
    ms = ctypes.c_float(0.0)
    rc = L.rtcc_gemm(PREC_TAG[prec], M, N, K, alpha, _p(ops.ar), _p(ops.ai), ops.lda, ta, _p(ops.br), _p(ops.bi),
                     ops.ldb, tb, beta, _p(ops.cr), _p(ops.ci), ops.ldc, ch, reps, ctypes.byref(ms),
                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        return None
    return ms.value if reps > 0 else 0.0


def candidates(prec, shape):
    M, N, K, ac, bc, ta, tb = shape
    out = []
    for mn, bk, _ in TILES:
        if mn == 128128 and prec == "fp64":
            continue
        for s in SPLITS:
            if s > 1 and (K // s < bk or K < 256):
                continue
            out.append((1, mn, bk, s))
    if prec == "bf16x3" and (ac or bc) and 2.0 * M * N * K >= 1e8:
        # the right-hand side runs its large products on three streams at once: a split grid is kept
        # within the library's own workgroup cap (160; 320 for the two-per-CU kernel) so that a product
        # timed alone does not win by taking CUs the other streams need
        for kern in (1, 2, 3, 4):  # register-staged, direct-to-LDS ring, the ring at two per CU, wide waves
            for wn in ((2,) if kern == 3 else (4,) if kern == 4 else (2, 4)):
                tiles = -(-M // 128) * -(-N // (64 * wn))
                for s in range(1, 17):
                    if s > 1 and (K // s < 64 or tiles * s > (320 if kern == 3 else 160)):
                        continue
                    out.append((2, wn, kern, s))
    return out


def shapes_to_tune(shapes, max_flops=0.0):
    """The (shape, call count) pairs to time, in a fixed order: all of them, or with max_flops > 0 only
    those with 2 M N K below max_flops (the table entries of the others stay as they are)."""
    return [(s, c) for s, c in sorted(shapes.items()) if max_flops <= 0 or 2.0 * s[0] * s[1] * s[2] < max_flops]


def load_entries(path):
    """The entries of an existing table by key (prec, M, N, K, ac, bc, ta, tb), each line kept verbatim
    (comment and malformed lines are dropped)."""
    keep = {}
    if os.path.exists(path):
        for line in open(path):
            body = line.split("#")[0].split()
            if len(body) == 12:
                keep[tuple(int(x) for x in body[:8])] = line.rstrip("\n")
    return keep


def tune_shape(L, prec, shape, target_ms=3.0):
    ops = Operands(*shape, prec)
    t0 = run_gemm(L, prec, ops, None, reps=3)
    reps = int(min(50, max(3, target_ms / max(t0, 1e-3))))
    base = run_gemm(L, prec, ops, None, reps=reps)
    best = (base, (0, 0, 0, 0))
    for c in candidates(prec, shape):
        t = run_gemm(L, prec, ops, c, reps=reps)
        if t is not None and t < best[0]:
            best = (t, c)
    return base, best


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--o", type=int, default=20)
    ap.add_argument("--v", type=int, default=76)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--min-gain", type=float, default=0.03)
    ap.add_argument("--batch", type=int, default=0, help="tune the products of a batched step of this many members")
    ap.add_argument("--max-flops", type=float, default=0.0,
                    help="tune only the products with 2 M N K below this (0: all); in the split-BF16 context 5e8 "
                         "selects the products that stay on the FP32 tile kernel")
    args = ap.parse_args()
    import torch
    from paper_2205_05175_amd import load_library
    L = load_library()
    L.rtcc_load_tuning(None, None)  # time the library's own rules, not an older table
    keep = load_entries(args.out)  # entries of other sizes stay
    total_gain = 0.0
    for prec in args.precisions.split(","):
        shapes = collect_shapes(args.o, args.v, prec, args.batch)
        print(f"[autotune] ({args.o},{args.v}) x{max(args.batch, 1)} {prec}: {len(shapes)} GEMM shapes", flush=True)
        for shape, count in shapes_to_tune(shapes, args.max_flops):
            t1 = time.time()
            base, (best_t, c) = tune_shape(L, prec, shape)
            M, N, K, ac, bc, ta, tb = shape
            key = (PREC_TAG[prec], M, N, K, int(ac), int(bc), ta, tb)
            gain = (base - best_t) / base if base else 0.0
            msg = (f"[autotune] {prec} M={M} N={N} K={K} {'c' if ac else 'r'}{'c' if bc else 'r'} ta={ta} tb={tb} "
                   f"x{count}: rule {1e3 * base:.1f} us, best {1e3 * best_t:.1f} us {c} ({time.time() - t1:.1f} s)")
            print(msg, flush=True)
            if c[0] != 0 and gain > args.min_gain:
                tag = f"({args.o},{args.v})" + (f" x{args.batch} members" if args.batch else "")
                keep[key] = (" ".join(str(x) for x in key) + " " + " ".join(str(x) for x in c) +
                             f"  # {tag}, {count} per call: {1e3 * best_t:.1f} us vs rule {1e3 * base:.1f} us")
                total_gain += count * (base - best_t)
            else:
                keep.pop(key, None)
        torch.cuda.synchronize()
    with open(args.out, "w") as fh:
        fh.write("# GEMM tuning table (paper_2205_05175_amd/autotune.py): prec M N K ac bc ta tb kind p1 p2 splits\n"
                 "# prec 0 FP64, 1 FP32, 2 split-BF16 contexts; kind 1 tile (p1 = bm*1000+bn, p2 = k stage),\n"
                 "# kind 2 split-BF16 (p1 = waves along N); times are per call, measured alone on random operands\n")
        for k in sorted(keep):
            fh.write(keep[k] + "\n")
    print(f"[autotune] wrote {len(keep)} entries to {args.out}; summed gain {1e3 * total_gain:.1f} us per RHS "
          f"(alone, all precisions)", flush=True)


if __name__ == "__main__":
    main()
