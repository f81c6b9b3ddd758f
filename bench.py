"""Benchmark: RK4 steps/s of real-time CCSD (T + Lambda right-hand side) at o=20, v=76 on one MI355X.

Workload (synthetic, seeded): the four-water-shaped closed-shell system o = 20 occupied and
v = 76 virtual spatial orbitals from ``synth.make_system(20, 76, seed=0)``; its FP64 ground
state is computed on the GPU, then a delta kick of 1e-3 au along z is applied, and the state
is propagated with RK4 at dt = 0.02 au. A timed "step" is one full RK4 step: four evaluations
of the T1/T2/Lambda1/Lambda2 time derivatives, the FP64 stage updates, and the FP64 dipole at
the step end. Both contraction precisions are timed on the same starting state; the headline
``value`` is the complex-FP32 path, ``fp64_steps_per_s`` the FP64 path.

The ladder GEMM (the dominant kernel) is timed live with HIP events recorded on the library's
stream around every launch inside the timed region. The CPU oracle is timed on a bounded
sample on the host (see ``cpu_baseline.sample``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}

# HBM bytes per launch of the split-BF16 ladder kernel (gemm_bf16x3_nt<1, 0, 1, 4>, o=20 v=76),
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the
# same counter on a plain device copy of the same run (the 72,247.5 KiB state clone: FETCH_SIZE
# 36,139.2 KiB, x2.0; WRITE_SIZE 72,247.5 KiB, x1.0). Commands and raw figures:
# profiles/ladder_traffic_o20v76.md. To be re-measured whenever that kernel changes.
LADDER_TRAFFIC_BF16X3 = {"fetch_bytes": 246305.8 * 1024 * 2.0, "write_bytes": 38464.0 * 1024 * 1.0,
                         "kernel": "gemm_bf16x3_nt<1, 0, 1, 4>"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline():
    """Oracle (spin-orbital FP64 NumPy) on the host: one RHS at (o,v) = (10,38), scaled to an RK4 step at (20,76)."""
    from oracle import ccsd
    from synth import make_system, random_state
    o, v = 10, 38
    eri, fock, mu = make_system(o, v, 0)
    S = ccsd.SpinOrbitalSystem(eri, fock, mu, o, v)
    st = random_state(o, v, 1)
    t0 = time.perf_counter()
    ccsd.rhs(S, *st, np.zeros(3))
    dt = time.perf_counter() - t0
    scale = (20 / 10) ** 2 * (76 / 38) ** 4  # o^2 v^4 ladder cost ratio
    step_s = 4 * dt * scale
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": 1.0 / step_s, "unit": "RK4 steps/s", "cores": threads, "kind": "oracle",
            "sample": f"one oracle RHS at (o,v)=(10,38) took {dt:.2f} s; x4 RHS per RK4 step and x{scale:.0f} "
                      f"(o^2 v^4 ratio to (20,76)); the full (20,76) spin-orbital oracle needs ~11 GB of "
                      f"antisymmetrised integrals and minutes per RHS"}


def bench_batch(args):
    """24 propagations in one captured step graph: 12 x (5,19) + 12 x (10,38), each system's
    members are delta kicks along x, y, z with kappa in {1e-3, 5e-3, 0.01, 0.05}; complex-FP32
    contractions, FP64 state, RK4 dt = 0.02. Timed against the same 24 propagations run one after
    another with the single-propagation path (its own captured step graph per system)."""
    import torch
    from paper_2205_05175_amd import RTCC, Field, propagate_batch
    from synth import make_system

    steps, warm, dt = args.steps, args.warmup, args.dt
    specs = [(5, 19), (10, 38)]
    kappas = [1e-3, 5e-3, 0.01, 0.05]
    members = [(d, k) for k in kappas for d in range(3)]
    systems, ys = [], []
    for o, v in specs:
        eri, fock, mu = make_system(o, v, 0)
        R = RTCC(eri, fock, mu, o, v, "fp32")
        g = R.new_state()
        e = R.ground_state(g, 1e-12, 200)
        y = torch.stack([g.clone() for _ in members])
        for m, (d, k) in enumerate(members):
            n = [0.0, 0.0, 0.0]
            n[d] = 1.0
            R.kick(y[m], k, n)
        systems.append(R)
        ys.append(y)
        log(f"[bench] batch system o={o} v={v}: e_corr={e:.10f}, {len(members)} kicked members")
    fields = [[Field.none() for _ in members] for _ in specs]
    nm = len(members)

    # batched: warm-up (captures the step graph), then the timed steps with dipoles recorded
    yb = [y.clone() for y in ys]
    propagate_batch(systems, yb, fields, 0.0, dt, warm, None)
    mus = [torch.zeros((steps + 1) * nm * 6, dtype=torch.float64, device="cuda") for _ in specs]
    torch.cuda.synchronize()
    ts = time.perf_counter()
    propagate_batch(systems, yb, fields, warm * dt, dt, steps, mus)
    torch.cuda.synchronize()
    tb = time.perf_counter() - ts
    log(f"[bench] batched: {steps} steps of {2 * nm} propagations in {tb:.3f} s")

    # ladder of the (10,38) system timed with HIP events (plain launches while profiling)
    R = systems[1]
    yp = [y.clone() for y in yb]
    pst = min(steps, 5)
    R.profile(True)
    propagate_batch(systems, yp, fields, (warm + steps) * dt, dt, pst, None)
    nl, ms, fl = R.profile_read()
    R.profile(False)
    del yp

    # sequential: the same 24 propagations one after another, each through a fixed state buffer
    # (so each system's captured step graph is reused), dipoles recorded
    mseq = []
    work = [R_.new_state() for R_ in systems]
    mw = torch.zeros((warm + 1, 6), dtype=torch.float64, device="cuda")
    for s, R_ in enumerate(systems):
        work[s].copy_(ys[s][0])
        R_.propagate_rk4(work[s], 0.0, dt, warm, None, mw)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s, R_ in enumerate(systems):
        for m in range(nm):
            work[s].copy_(ys[s][m])
            R_.propagate_rk4(work[s], 0.0, dt, warm, None, mw)
            mo = torch.zeros((steps + 1, 6), dtype=torch.float64, device="cuda")
            R_.propagate_rk4(work[s], warm * dt, dt, steps, None, mo)
            mseq.append(mo)
    torch.cuda.synchronize()
    tsq = time.perf_counter() - ts
    log(f"[bench] sequential: {2 * nm} propagations x {warm + steps} steps in {tsq:.3f} s")
    tsq_timed = tsq * steps / (warm + steps)  # the warm-up steps of each member are not part of the comparison
    err = 0.0
    for s in range(len(specs)):
        mb = mus[s].view(steps + 1, nm, 6).cpu().numpy()
        for m in range(nm):
            err = max(err, float(np.abs(mb[:, m] - mseq[s * nm + m].cpu().numpy()).max()))
    member_steps = 2 * nm * steps
    avg = ms / max(nl, 1)
    tfl = fl / (avg * 1e-3) / 1e12 if nl else 0.0
    line = {
        "metric": "batched RK4 member-steps/s: 24 propagations (12 x (5,19) + 12 x (10,38)) in one captured graph",
        "value": member_steps / tb, "unit": "member RK4 steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": 1e3 * tb / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched rt-ccsd: synthetic water-shaped (5,19) and (10,38) seed 0, 12 delta kicks "
                               "each (x/y/z x kappa 1e-3, 5e-3, 0.01, 0.05), RK4 dt=0.02",
                   "members": 2 * nm, "precision": "complex fp32 contractions, fp64 state",
                   "parallelism": "single GPU"},
        "sequential_member_steps_per_s": member_steps / tsq_timed,
        "speedup_vs_sequential": tsq_timed / tb,
        "dipole_batch_vs_sequential_max_abs": err,
        "roofline": {"bound": "mfma", "kernel": "batched ladder GEMM of the (10,38) system (12 members, fp32)",
                     "achieved": tfl, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s", "frac": tfl / PEAK_TFLOPS["fp32"],
                     "traffic": None, "avg_ms": avg, "flops_per_launch": fl},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_adjoint(args):
    """Gradient of L = dt * trapezoid(Re mu_z) over 200 RK4 steps (dt = 0.05) at (10,38) with respect
    to the Gaussian pulse (E0, omega, sigma, t0) = (0.01, 0.5, 5, 15) along z: complex-FP32 forward
    with segment checkpoints every 20 steps, then the adjoint sweep (FP64 adjoint state). Checked
    against central differences (h = 1e-5) of the GPU FP64 loss."""
    import torch
    from paper_2205_05175_amd import RTCC, Field
    from paper_2205_05175_amd.adjoint import integrated_dipole, pulse_dipole_trajectory
    from synth import make_system

    o, v, dt, N, every = 10, 38, 0.05, args.steps, 20
    n = [0.0, 0.0, 1.0]
    p0 = np.array([0.01, 0.5, 5.0, 15.0])
    eri, fock, mu = make_system(o, v, 0)
    R = RTCC(eri, fock, mu, o, v, "fp32")
    y0 = R.new_state()
    R.set_precision("fp64")
    R.ground_state(y0, 1e-12, 200)
    R.set_precision("fp32")

    def grad_once():
        params = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        L = integrated_dipole(pulse_dipole_trajectory(R, params, y0, n, 0.0, dt, N, every=every), dt)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        return params.grad.numpy().copy(), L.item(), tb - ta, tc - tb

    for _ in range(max(args.warmup, 1)):
        grad_once()
    reps = 3
    runs = [grad_once() for _ in range(reps)]
    g, L, tf, tbk = runs[-1]
    tf = min(r[2] for r in runs)
    tbk = min(r[3] for r in runs)
    log(f"[bench] adjoint: forward {tf:.3f} s, backward {tbk:.3f} s, grad {g}")

    def loss64(pp):
        R.set_precision("fp64")
        y = y0.clone()
        m = torch.zeros((N + 1, 6), dtype=torch.float64, device="cuda")
        R.propagate_rk4(y, 0.0, dt, N, Field.gaussian(*pp, n), m)
        x = m[:, 4].cpu().numpy()
        return dt * (x.sum() - 0.5 * (x[0] + x[-1]))

    fd = np.zeros(4)
    for j in range(4):
        st = 1e-5 * (1.0 if j == 0 else abs(p0[j]))
        e = np.zeros(4)
        e[j] = st
        fd[j] = (loss64(p0 + e) - loss64(p0 - e)) / (2 * st)
    R.set_precision("fp32")
    err = float(np.abs(g - fd).max() / np.abs(fd).max())
    line = {
        "metric": "adjoint gradient of the time-integrated dipole w.r.t. the pulse parameters, (10,38), 200 RK4 steps",
        "value": 1.0 / (tf + tbk), "unit": "gradients/s", "n_gpus": 1, "steps": N, "warmup": args.warmup,
        "ms_per_step": 1e3 * (tf + tbk) / N, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rt-ccsd adjoint: synthetic water-shaped (10,38) seed 0, Gaussian pulse E0=0.01 "
                               "omega=0.5 sigma=5 t0=15 along z, RK4 dt=0.05, loss dt*trapz(Re mu_z), "
                               "checkpoints every 20 steps",
                   "precision": "complex fp32 contractions, fp64 state and adjoint", "parallelism": "single GPU"},
        "forward_s": tf, "backward_s": tbk, "backward_over_forward": tbk / tf,
        "gradient": g.tolist(), "fd_gradient_fp64": fd.tolist(), "max_rel_err_vs_fd": err,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["single", "batch", "adjoint"], default="single",
                    help="single: the o=20 v=76 propagation (default); batch: 24 batched propagations; "
                         "adjoint: pulse-parameter gradient at (10,38)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--o", type=int, default=20)
    ap.add_argument("--v", type=int, default=76)
    ap.add_argument("--dt", type=float, default=0.02)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library evaluates each "
              f"propagation on a single GPU; independent propagations are batched on that GPU instead",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        if args.steps is None:
            args.steps = 500
        return bench_batch(args)
    if args.workload == "adjoint":
        if args.steps is None:
            args.steps = 200
        return bench_adjoint(args)
    if args.steps is None:
        args.steps = 20

    import torch
    from paper_2205_05175_amd import RTCC
    from synth import make_system

    o, v = args.o, args.v
    t0 = time.time()
    eri, fock, mu = make_system(o, v, 0)
    log(f"[bench] system o={o} v={v} built in {time.time() - t0:.1f} s")
    R = RTCC(eri, fock, mu, o, v, precision="fp32")
    del eri
    y0 = R.new_state()
    t0 = time.time()
    e_corr = R.ground_state(y0, 1e-10, 200)
    torch.cuda.synchronize()
    log(f"[bench] ground state e_corr={e_corr:.12f} in {time.time() - t0:.1f} s")
    R.kick(y0, 1e-3, [0.0, 0.0, 1.0])

    results = {}
    finals = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        R.set_precision(prec)
        y = y0.clone()
        # warm-up builds the captured step graph before the timed region
        mu_w = torch.zeros((args.warmup + 1, 6), dtype=torch.float64, device="cuda")
        R.propagate_rk4(y, 0.0, args.dt, args.warmup, None, mu_w)
        mu_t = torch.zeros((args.steps + 1, 6), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        R.propagate_rk4(y, args.warmup * args.dt, args.dt, args.steps, None, mu_t)
        torch.cuda.synchronize()
        te = time.perf_counter()
        # ladder-GEMM timing: the same steps again with HIP events around every ladder launch
        # (events cannot be timed inside a captured graph, so this pass issues plain launches)
        yp = y.clone()
        mu_p = torch.zeros((args.steps + 1, 6), dtype=torch.float64, device="cuda")
        R.profile(True)
        tp0 = time.perf_counter()
        R.propagate_rk4(yp, (args.warmup + args.steps) * args.dt, args.dt, args.steps, None, mu_p)
        n, ms, fl = R.profile_read()
        tp1 = time.perf_counter()
        R.profile(False)
        del yp, mu_p
        bad = R.check_state(y)
        if bad:
            raise SystemExit(f"non-finite state after {prec} propagation ({bad} entries)")
        avg = ms / max(n, 1)
        results[prec] = {"ms_per_step": 1e3 * (te - ts) / args.steps, "steps_per_s": args.steps / (te - ts),
                         "eager_ms_per_step": 1e3 * (tp1 - tp0) / args.steps,
                         "ladder_launches": n, "ladder_ms": avg, "ladder_flops": fl,
                         "ladder_tflops": fl / (avg * 1e-3) / 1e12 if n else 0.0}
        finals[prec] = (y, mu_t.cpu().numpy())
        log(f"[bench] {prec}: {results[prec]}")

    # dipole checks: FP32 vs FP64 trajectories, and the GPU dipole of the final FP64 state vs the oracle
    cm = lambda m: m[:, 0::2] + 1j * m[:, 1::2]
    m64 = cm(finals["fp64"][1])
    fp32_err = float(np.abs(cm(finals["fp32"][1]) - m64).max())
    bf16_err = float(np.abs(cm(finals["bf16x3"][1]) - m64).max())
    from oracle import ccsd
    from synth import unpack_state
    S = ccsd.SpinOrbitalSystem(None, fock, mu, o, v)
    yf = finals["fp64"][0].cpu().numpy()
    mu_oracle = ccsd.dipole(S, *unpack_state(yf, o, v))
    oracle_err = float(np.abs(R.dipole(finals["fp64"][0]) - mu_oracle).max())

    cpu = None if args.no_cpu else cpu_baseline()
    r32 = results["fp32"]
    rbf = results["bf16x3"]
    # the headline path is split-BF16 when its dipole stays within 1e-6 au of FP64, else complex FP32
    head = "bf16x3" if bf16_err <= 1e-6 else "fp32"
    rh = results[head]
    measured_traffic = head == "bf16x3" and (o, v) == (20, 76)
    line = {
        "metric": "RK4 steps/s (T+Λ RHS) o=20,v=76: FP32-MFMA vs FP64, dipole err vs oracle",
        "value": rh["steps_per_s"], "unit": "RK4 steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rh["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3" if head == "bf16x3" else "f32", "data": "synthetic",
        "config": {"workload": f"rt-ccsd four-water-shaped synthetic o={o} v={v} seed 0, delta kick 1e-3 z, "
                               f"RK4 dt={args.dt}", "o": o, "v": v,
                   "precision": ("split-bf16 three-term products (complex, fp32 accumulate) on products above "
                                 "5e8 flop, fp32 elsewhere, fp64 state" if head == "bf16x3" else
                                 "complex fp32 contractions, fp64 state"), "parallelism": "single GPU"},
        "headline_path": head,
        "fp64_steps_per_s": results["fp64"]["steps_per_s"],
        "fp32_steps_per_s": r32["steps_per_s"],
        "bf16x3_steps_per_s": rbf["steps_per_s"],
        "fp32_over_fp64": r32["steps_per_s"] / results["fp64"]["steps_per_s"],
        "bf16x3_over_fp64": rbf["steps_per_s"] / results["fp64"]["steps_per_s"],
        "dipole_fp32_vs_fp64_max_abs": fp32_err,
        "dipole_bf16x3_vs_fp64_max_abs": bf16_err,
        "dipole_fp64_gpu_vs_oracle_max_abs": oracle_err,
        "roofline": {"bound": "mfma", "kernel": f"ladder GEMM ({head})", "achieved": rh["ladder_tflops"],
                     "peak": PEAK_TFLOPS["fp32"] if head == "fp32" else PEAK_TFLOPS["bf16"] / 3,
                     "unit": "TFLOP/s",
                     "frac": rh["ladder_tflops"] / (PEAK_TFLOPS["fp32"] if head == "fp32" else PEAK_TFLOPS["bf16"] / 3),
                     "peak_note": ("fp32 MFMA peak" if head == "fp32" else "bf16 dense MFMA peak / 3 products per "
                                   "real multiply (algorithmic fp32-equivalent flops)"),
                     "traffic": (LADDER_TRAFFIC_BF16X3["fetch_bytes"] + LADDER_TRAFFIC_BF16X3["write_bytes"]
                                 if measured_traffic else None),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     # packed operands read once (X: 896 x 5792 x 4 bf16 planes, V: 5888 x 5792 x 2) and
                     # the 800 x 5776 complex FP32 output written once (one K split at this size)
                     "traffic_algorithmic_min": (2 * 896 * 5792 * 4 + 2 * 5888 * 5792 * 2 + 800 * 5776 * 8
                                                 if measured_traffic else None),
                     "avg_ms": rh["ladder_ms"], "flops_per_launch": rh["ladder_flops"],
                     "fp32": {"achieved": r32["ladder_tflops"], "peak": PEAK_TFLOPS["fp32"],
                              "frac": r32["ladder_tflops"] / PEAK_TFLOPS["fp32"], "avg_ms": r32["ladder_ms"]},
                     "fp64": {"achieved": results["fp64"]["ladder_tflops"], "peak": PEAK_TFLOPS["fp64"],
                              "frac": results["fp64"]["ladder_tflops"] / PEAK_TFLOPS["fp64"],
                              "avg_ms": results["fp64"]["ladder_ms"]}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
