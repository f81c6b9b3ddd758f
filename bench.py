"""Benchmark: RK4 steps/s of real-time CCSD (T + Lambda right-hand side) at o=20, v=76 on one MI355X.

Workload (synthetic, seeded): the four-water-shaped closed-shell system o = 20 occupied and
v = 76 virtual spatial orbitals from ``synth.make_system(20, 76, seed=0)`` (factor width
0.05 * 24 / n: the unscaled width of the smaller systems has no convergent CCSD solution at this
size); its FP64 ground state is computed on the GPU, then a delta kick of 1e-3 au along z is
applied, and the state is propagated with RK4 at dt = 0.02 au. A timed "step" is one full RK4
step: four evaluations of the T1/T2/Lambda1/Lambda2 time derivatives, the FP64 stage updates,
and the FP64 dipole at the step end. FP64, complex-FP32 and split-BF16 contractions are timed on
the same starting state. The headline ``value`` is the split-BF16 path when its dipole stays
within 1e-6 au of the FP64 path over the whole gate trajectory (``--gate-steps`` RK4 steps from
the kick, 500 by default), else the complex-FP32 path.

The dominant kernel -- the large complex x complex products of the ring and Lambda terms, in the
split-BF16 path the register-staged kernel gemm_bf16x3_nt<1, 1, 0, 4> -- is timed live with HIP
events recorded on the stream each launch runs on, around every launch of a second, eagerly issued
pass of the timed steps (``roofline``); the ladder GEMMs likewise in a third pass
(``ladder_roofline``). The CPU oracle is timed on a bounded sample on the host (see
``cpu_baseline.sample``).

Other workloads: ``--workload spectrum`` (RK4 and adaptive Cash-Karp to t = 100 au in every
precision, absorption-peak shifts against FP64), ``sp-spectra`` (the paper's narrow-pulse double- vs
single-precision spectra at (5,19) and (10,38) to t = 300 au, and the dipole noise-injection study),
``integrators`` (RK4, Cash-Karp, Fehlberg 4(5) and implicit Gauss-Legendre on the (20,76) propagation:
right-hand sides and dipole error against a finer RK4),
``batch`` (24 propagations in one captured graph per step), ``adjoint`` (pulse-parameter gradient at
(10,38)).
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
# 36,150.1 KiB, x2.0; WRITE_SIZE 72,248.4 KiB, x1.0). Commands and raw figures:
# profiles/ladder_traffic_o20v76.md. To be re-measured whenever that kernel changes. It applies to the
# full ladder product (RTCC_LADDER=full).
LADDER_TRAFFIC_BF16X3 = {"fetch_bytes": 246317.7 * 1024 * 2.0, "write_bytes": 38517.8 * 1024 * 1.0,
                         "kernel": "gemm_bf16x3_nt<1, 0, 1, 4>"}
# The same for the symmetric / antisymmetric ladder (the default): its two GEMMs (X+V+: 420 x 2926 x 2926,
# X-V-: 380 x 2850 x 2850, 3 K splits each) in one launch of gemm_bf16x3_nt2<1, 0, 1, 4>, in the RK4 step of
# bench.py --workload profile (FETCH_SIZE 73,664.2 KiB, WRITE_SIZE 69,977.8 KiB per dispatch; the same
# run's state clone: FETCH_SIZE x2.0, WRITE_SIZE x1.0). Commands: profiles/ladder_traffic_o20v76.md.
LADDER_TRAFFIC_BF16X3_SYM = {"fetch_bytes": 73664.2 * 1024 * 2.0, "write_bytes": 69977.8 * 1024 * 1.0,
                             "kernel": "gemm_bf16x3_nt2<1, 0, 1, 4>"}
# The dominant kernel of the split-BF16 step, the register-staged complex x complex kernel
# gemm_bf16x3_nt<1, 1, 0, 4> (the ring and Lambda products, 12 launches per right-hand side at o=20
# v=76, three of them carrying three independent products each): mean HBM bytes per dispatch over its
# launches in the RK4 step of bench.py --workload profile, calibrated on the same run's state clone like
# the ladder's (FETCH_SIZE 59,570.3 KiB x2.0, WRITE_SIZE 37,188.1 KiB x1.0 per dispatch, 144 dispatches).
# Commands: profiles/cc_gemm_o20v76.md.
CC_TRAFFIC_BF16X3 = {"fetch_bytes": 59570.3 * 1024 * 2.0, "write_bytes": 37188.1 * 1024 * 1.0,
                     "kernel": "gemm_bf16x3_nt<1, 1, 0, 4>"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline_leg(fock, mu, o, v, y64_final, gpu_dipole):
    """The oracle on the host cores: timed as planned (medians of 3 right-hand sides at (4,16),
    (5,19) and (10,38), of 3 RK4 steps at (4,16) and (5,19), one RK4 step at (10,38)), the RK4 step
    rate extrapolated to (o, v) by the o^2 v^4 ladder cost, and the FP64 GPU dipole of the final
    state checked against the oracle's dipole at full size (the dipole needs no two-electron
    integrals)."""
    from oracle import ccsd, integrators
    from synth import make_system, pack_state, random_state, unpack_state
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rows, t_all = [], time.perf_counter()
    rk4_1038 = None
    for (so, sv), n_rhs, n_step in (((4, 16), 3, 3), ((5, 19), 3, 3), ((10, 38), 3, 1)):
        eri, fk, mm = make_system(so, sv, 0)
        S = ccsd.SpinOrbitalSystem(eri, fk, mm, so, sv)
        st = random_state(so, sv, 1)
        E = np.zeros(3)
        tr = []
        for _ in range(n_rhs):
            t0 = time.perf_counter()
            ccsd.rhs(S, *st, E)
            tr.append(time.perf_counter() - t0)
        f = lambda t, yy: pack_state(*ccsd.rhs(S, *unpack_state(yy, so, sv), E))
        y = pack_state(*st)
        ts = []
        for _ in range(n_step):
            t0 = time.perf_counter()
            integrators.rk4_step(f, 0.0, y, 0.02)
            ts.append(time.perf_counter() - t0)
        rows.append({"o": so, "v": sv, "rhs_s_median": float(np.median(tr)), "rk4_step_s_median": float(np.median(ts)),
                     "rhs_samples": n_rhs, "rk4_samples": n_step})
        if (so, sv) == (10, 38):
            rk4_1038 = float(np.median(ts))
        del S, eri
    elapsed = time.perf_counter() - t_all
    scale = (o / 10) ** 2 * (v / 38) ** 4
    S = ccsd.SpinOrbitalSystem(None, fock, mu, o, v)
    mu_oracle = ccsd.dipole(S, *unpack_state(y64_final, o, v))
    dip_err = float(np.abs(gpu_dipole - mu_oracle).max())
    cpu = {"value": 1.0 / (rk4_1038 * scale), "unit": "RK4 steps/s", "cores": threads, "kind": "oracle",
           "extrapolated": True,
           "sample": (f"oracle (spin-orbital FP64 NumPy) on {threads} host threads, {elapsed:.1f} s in all: medians of "
                      f"3 RHS at (4,16), (5,19), (10,38), of 3 RK4 steps at (4,16), (5,19) and one RK4 step at "
                      f"(10,38) ({rk4_1038:.2f} s); value = that step extrapolated to (o,v)=({o},{v}) by the "
                      f"o^2 v^4 ladder cost (x{scale:.0f}); one oracle RHS at (20,76) needs ~11 GB of "
                      f"antisymmetrised integrals and is not part of this bounded sample"),
           "measured": rows}
    return cpu, dip_err


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
    nl, ms, fl, _ = R.profile_read()
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


def _propagate_chunked(R, y, t0, dt, nsteps, mu_full, k0, chunk, label):
    """nsteps RK4 steps from t0 with the dipole written to mu_full[k0 .. k0 + nsteps] (rows of 6),
    issued in chunks so that progress is printed while the GPU works."""
    import torch
    done = 0
    while done < nsteps:
        n = min(chunk, nsteps - done)
        R.propagate_rk4(y, t0 + done * dt, dt, n, None, mu_full[k0 + done:k0 + done + n + 1])
        torch.cuda.synchronize()
        done += n
        log(f"[bench] {label}: {done}/{nsteps} steps")


def bench_spectrum(args):
    """The o=20, v=76 delta-kick propagation to t = 100 au in every contraction precision: RK4 at
    dt = 0.02 (5000 steps) and adaptive Cash-Karp at eps = 1e-6; whole-trajectory dipole errors and
    absorption-peak shifts against the FP64 RK4 trajectory, and the Cash-Karp / RK4 count of
    right-hand sides."""
    import torch
    from paper_2205_05175_amd import RTCC
    from paper_2205_05175_amd import spectrum as spc
    from synth import make_system

    o, v, dt, T, kappa, eps = args.o, args.v, args.dt, args.t_end, 1e-3, args.eps
    nsteps = int(round(T / dt))
    eri, fock, mu = make_system(o, v, 0)
    R = RTCC(eri, fock, mu, o, v, precision="fp32")
    del eri
    y0 = R.new_state()
    R.set_precision("fp64")
    e_corr = R.ground_state(y0, 1e-10, 200)
    mu_gs = R.dipole(y0)
    R.kick(y0, kappa, [0.0, 0.0, 1.0])
    log(f"[bench] spectrum workload o={o} v={v}: e_corr={e_corr:.10f}, RK4 {nsteps} steps, CK eps={eps}")
    rk, ck = {}, {}
    for prec in ("fp64", "fp32", "bf16x3"):
        R.set_precision(prec)
        y = y0.clone()
        m = torch.zeros((nsteps + 1, 6), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _propagate_chunked(R, y, 0.0, dt, nsteps, m, 0, 500, f"rk4 {prec}")
        te = time.perf_counter() - ts
        bad = R.check_state(y)
        mm = m.cpu().numpy()
        rk[prec] = {"mu": mm[:, 0::2] + 1j * mm[:, 1::2], "s": te, "nonfinite": bad}
    sweep = {}
    for eps_k in [float(x) for x in args.eps_sweep.split(",") if x]:
        R.set_precision("bf16x3")
        y = y0.clone()
        t, h, nacc, nrej, times, mus = 0.0, 0.02, 0, 0, [0.0], [R.dipole(y)]
        ts = time.perf_counter()
        while t < T - 1e-12:
            t1 = min(T, t + 10.0)
            tt, mm, na, nr, h = R.propagate_cashkarp(y, t, t1, h, eps_k, cap=200000)
            times += list(tt)
            mus += list(mm)
            nacc, nrej, t = nacc + na, nrej + nr, t1
        log(f"[bench] cash-karp sweep eps={eps_k}: {nacc} accepted, {nrej} rejected")
        sweep[eps_k] = {"t": np.array(times), "mu": np.array(mus), "acc": nacc, "rej": nrej,
                        "s": time.perf_counter() - ts}
    for prec in ("fp64", "fp32", "bf16x3"):
        R.set_precision(prec)
        y = y0.clone()
        t, h = 0.0, 0.02
        times, mus, nacc, nrej = [0.0], [R.dipole(y)], 0, 0
        torch.cuda.synchronize()
        ts = time.perf_counter()
        while t < T - 1e-12:
            t1 = min(T, t + 10.0)
            tt, mm, na, nr, h = R.propagate_cashkarp(y, t, t1, h, eps, cap=200000)
            times += list(tt)
            mus += list(mm)
            nacc += na
            nrej += nr
            t = t1
            log(f"[bench] cash-karp {prec}: t = {t:.1f}, {nacc} accepted, {nrej} rejected")
        te = time.perf_counter() - ts
        ck[prec] = {"t": np.array(times), "mu": np.array(mus), "acc": nacc, "rej": nrej, "s": te}

    def induced(mz):
        return mz.real - mu_gs[2].real

    grid = dt * np.arange(nsteps + 1)
    ref = induced(rk["fp64"]["mu"][:, 2])
    out = {"rk4": {}, "cashkarp": {}}
    for prec in ("fp64", "fp32", "bf16x3"):
        r = rk[prec]
        cmp, p_ref, p_oth = spc.compare_trajectories(ref, induced(r["mu"][:, 2]), dt, kappa)
        out["rk4"][prec] = {"steps_per_s": nsteps / r["s"], "wall_s": r["s"], "nonfinite": r["nonfinite"],
                            "dipole_max_abs_vs_fp64": float(np.abs(r["mu"] - rk["fp64"]["mu"]).max()),
                            "peak_shift_max_vs_fp64": cmp.max_shift, "peaks_matched": len(cmp.pairs),
                            "unmatched_fp64": cmp.unmatched_ref, "unmatched": cmp.unmatched_other}
        c = ck[prec]
        tg, dz = spc.resample_uniform(c["t"], induced(c["mu"][:, 2]), dt, t_end=T)
        n = min(tg.size, grid.size)
        cmpc, _, _ = spc.compare_trajectories(ref[:n], dz[:n], dt, kappa)
        c64 = ck["fp64"]
        _, dz64 = spc.resample_uniform(c64["t"], induced(c64["mu"][:, 2]), dt, t_end=T)
        cmpp, _, _ = spc.compare_trajectories(dz64[:n], dz[:n], dt, kappa)
        same_steps = c["t"].size == c64["t"].size and bool(np.abs(c["t"] - c64["t"]).max() < 1e-9)
        out["cashkarp"][prec] = {"accepted": c["acc"], "rejected": c["rej"], "rhs": 6 * (c["acc"] + c["rej"]),
                                 "wall_s": c["s"], "rhs_ratio_rk4_over_ck": 4 * nsteps / (6 * (c["acc"] + c["rej"])),
                                 "speedup_vs_rk4_same_precision": r["s"] / c["s"],
                                 "mean_h": T / max(c["acc"], 1),
                                 "same_steps_as_fp64_ck": same_steps,
                                 "dipole_max_abs_vs_fp64_ck": (float(np.abs(c["mu"] - c64["mu"]).max())
                                                               if same_steps else None),
                                 "peak_shift_max_vs_fp64_ck": cmpp.max_shift, "unmatched_vs_fp64_ck":
                                     cmpp.unmatched_ref + cmpp.unmatched_other,
                                 "dipole_max_abs_vs_fp64_rk4_on_grid": float(np.abs(dz[:n] - ref[:n]).max()),
                                 "peak_shift_max_vs_fp64_rk4": cmpc.max_shift, "peaks_matched": len(cmpc.pairs),
                                 "unmatched_fp64": cmpc.unmatched_ref, "unmatched": cmpc.unmatched_other}
    out["cashkarp_eps_sweep_bf16x3"] = {}
    for eps_k, c in sweep.items():
        tg, dz = spc.resample_uniform(c["t"], induced(c["mu"][:, 2]), dt, t_end=T)
        n = min(tg.size, grid.size)
        cm, _, _ = spc.compare_trajectories(ref[:n], dz[:n], dt, kappa)
        out["cashkarp_eps_sweep_bf16x3"][str(eps_k)] = {
            "accepted": c["acc"], "rejected": c["rej"], "rhs": 6 * (c["acc"] + c["rej"]), "wall_s": c["s"],
            "rhs_ratio_rk4_over_ck": 4 * nsteps / (6 * (c["acc"] + c["rej"])),
            "dipole_max_abs_vs_fp64_rk4_on_grid": float(np.abs(dz[:n] - ref[:n]).max()),
            "peak_shift_max_vs_fp64_rk4": cm.max_shift, "unmatched": cm.unmatched_ref + cm.unmatched_other}
    w, S64 = spc.absorption(ref, dt, kappa)
    peaks = [p.omega for p in spc.find_peaks(w, S64)]
    head = out["rk4"]["bf16x3"]
    line = {
        "metric": "absorption-peak shift vs FP64 (RK4 dt=0.02 and Cash-Karp eps=1e-6 to t=100 au), o=20 v=76",
        "value": max(out["rk4"]["fp32"]["peak_shift_max_vs_fp64"], head["peak_shift_max_vs_fp64"]),
        "unit": "Eh", "n_gpus": 1, "steps": nsteps, "warmup": 0, "ms_per_step": 1e3 / head["steps_per_s"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32/bf16x3", "data": "synthetic",
        "config": {"workload": f"rt-ccsd four-water-shaped synthetic o={o} v={v} seed 0 (factor width 0.05*24/n), "
                               f"delta kick {kappa} z, RK4 dt={dt} and Cash-Karp eps={eps} to t={T} au",
                   "parallelism": "single GPU"},
        "fp64_peaks_Eh": peaks,
        "rk4": out["rk4"], "cashkarp": out["cashkarp"], "cashkarp_eps_sweep_bf16x3": out["cashkarp_eps_sweep_bf16x3"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_sp_spectra(args):
    """Double- vs single-precision spectra with the paper's narrow pulse (Results, single precision):
    E0 = 0.01 au, nu = 0.05 au, sigma = 0.01 au, no carrier, isotropic n, RK4 at h = 0.01 au to
    t = 300 au, for each synthetic size in --sizes and every contraction precision; then the noise
    study on the FP64 trajectory (uniform noise of magnitude 1e-9 ... 1e-3 au added to the dipole)."""
    import torch
    from paper_2205_05175_amd import RTCC, Field
    from paper_2205_05175_amd import spectrum as spc
    from synth import make_system

    dt, T = args.dt, args.t_end
    E0, nu, sigma = 0.01, 0.05, 0.01
    n_iso = np.ones(3) / np.sqrt(3.0)
    kappa = -E0 * sigma * np.sqrt(2.0 * np.pi)  # integral of the pulse: the equivalent kick
    nsteps = int(round(T / dt))
    mags = [10.0 ** k for k in range(-9, -2)]
    sizes = [tuple(int(x) for x in s.split("x")) for s in args.sizes.split(",") if s]
    out = {}
    for o, v in sizes:
        eri, fock, mu = make_system(o, v, 0)
        R = RTCC(eri, fock, mu, o, v, precision="fp32")
        del eri
        y0 = R.new_state()
        R.set_precision("fp64")
        R.ground_state(y0, 1e-10, 200)
        d_gs = float(np.dot(n_iso, R.dipole(y0).real))
        fld = Field.gaussian(E0, 0.0, sigma, nu, n_iso)
        traj = {}
        for prec in ("fp64", "fp32", "bf16x3"):
            R.set_precision(prec)
            y = y0.clone()
            m = torch.zeros((nsteps + 1, 6), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            ts = time.perf_counter()
            done = 0
            while done < nsteps:
                n = min(2000, nsteps - done)
                R.propagate_rk4(y, done * dt, dt, n, fld, m[done:done + n + 1])
                torch.cuda.synchronize()
                done += n
                log(f"[bench] sp-spectra ({o},{v}) {prec}: {done}/{nsteps} steps")
            te = time.perf_counter() - ts
            mm = m.cpu().numpy()
            traj[prec] = {"d": mm[:, 0::2] @ n_iso - d_gs, "s": te, "nonfinite": R.check_state(y)}
        R.close()
        # samples at t_k = k dt, the pulse centred at nu: time origin of the response at the pulse
        d64 = traj["fp64"]["d"]
        w, s64 = spc.absorption(d64, dt, kappa, t0=-nu)
        p64 = spc.find_peaks(w, s64)
        res = {"fp64_peaks_Eh": [p.omega for p in p64], "steps_per_s": {}, "vs_fp64": {}}
        for prec, tr in traj.items():
            res["steps_per_s"][prec] = nsteps / tr["s"]
            if prec == "fp64":
                continue
            _, sp_ = spc.absorption(tr["d"], dt, kappa, t0=-nu)
            c = spc.match_peaks(p64, spc.find_peaks(w, sp_))
            res["vs_fp64"][prec] = {"dipole_max_abs": float(np.abs(tr["d"] - d64).max()),
                                    "peak_shift_max": c.max_shift, "peaks_matched": len(c.pairs),
                                    "unmatched": c.unmatched_ref + c.unmatched_other,
                                    "nonfinite": tr["nonfinite"]}
        study = spc.noise_study(d64, dt, kappa, mags, seed=0, t0=-nu)
        res["noise_study_fp64"] = [{"magnitude": r.magnitude, "unchanged": r.unchanged,
                                    "peak_shift_max": r.comparison.max_shift,
                                    "unmatched": len(r.comparison.unmatched_ref) + len(r.comparison.unmatched_other),
                                    "low_freq_peaks": r.low_freq_peaks, "max_rel_change": r.max_rel_change}
                                   for r in study]
        res["first_noise_magnitude_that_loses_peaks"] = next((r.magnitude for r in study if not r.unchanged), None)
        res["first_noise_magnitude_shifting_peaks_over_1e-4_Eh"] = next(
            (r.magnitude for r in study if r.comparison.max_shift > 1e-4 or not r.unchanged), None)
        res["induced_dipole_max_abs"] = float(np.abs(d64).max())
        out[f"{o}x{v}"] = res
    worst = max(r["vs_fp64"][p]["peak_shift_max"] for r in out.values() for p in ("fp32", "bf16x3"))
    line = {
        "metric": "absorption-peak shift, single vs double precision (paper's narrow pulse, RK4 h=0.01 to t=300 au)",
        "value": worst, "unit": "Eh", "n_gpus": 1, "steps": nsteps, "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/bf16x3", "data": "synthetic",
        "config": {"workload": f"rt-ccsd water-cluster-shaped synthetic {args.sizes} seed 0, Gaussian pulse E0={E0} "
                               f"nu={nu} sigma={sigma} au along (1,1,1)/sqrt3, RK4 h={dt} to t={T} au; noise study "
                               f"on the FP64 dipole (uniform, magnitudes 1e-9..1e-3 au)",
                   "parallelism": "single GPU"},
        "sizes": out, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_integrators(args):
    """The integrators of the tableau engine on the o=20, v=76 delta-kick propagation (split-BF16
    contractions): RK4 at h = dt, adaptive Cash-Karp and Fehlberg 4(5) at eps, implicit Gauss-Legendre
    with two and three stages at larger steps; right-hand sides, wall time and the largest dipole
    deviation from RK4 at h = dt / 2 (the reference, splined onto every integrator's sample times)."""
    import torch
    from scipy.interpolate import CubicSpline
    from paper_2205_05175_amd import RTCC
    from synth import make_system

    o, v, dt, T, eps = args.o, args.v, args.dt, args.t_end, args.eps
    eri, fock, mu = make_system(o, v, 0)
    R = RTCC(eri, fock, mu, o, v, precision="bf16x3")
    del eri
    y0 = R.new_state()
    R.set_precision("fp64")
    R.ground_state(y0, 1e-10, 200)
    R.kick(y0, 1e-3, [0.0, 0.0, 1.0])
    R.set_precision("bf16x3")
    log(f"[bench] integrators workload o={o} v={v}: t_end={T}, RK4 dt={dt}, eps={eps}")

    def rk4(h):
        n = int(round(T / h))
        y = y0.clone()
        m = torch.zeros((n + 1, 6), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _propagate_chunked(R, y, 0.0, h, n, m, 0, 500, f"rk4 h={h}")
        te = time.perf_counter() - ts
        return h * np.arange(n + 1), m.cpu().numpy()[:, 4], 4 * n, te

    tref, mref, _, _ = rk4(dt / 2)
    ref = CubicSpline(tref, mref)
    res = {}
    t_, m_, rhs, te = rk4(dt)
    res[f"rk4 h={dt}"] = {"rhs": rhs, "wall_s": te, "accepted": len(t_) - 1, "rejected": 0,
                         "dipole_max_abs_vs_ref": float(np.abs(m_ - ref(t_)).max())}
    for e in (eps, eps / 100):
        for name in ("cashkarp", "rkf45"):
            y = y0.clone()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            tt, mm, na, nr, _ = R.propagate_embedded(y, 0.0, T, dt, e, name)
            te = time.perf_counter() - ts
            res[f"{name} eps={e:g}"] = {"rhs": 6 * (na + nr), "wall_s": te, "accepted": na, "rejected": nr,
                                        "dipole_max_abs_vs_ref": float(np.abs(mm[:, 2].real - ref(tt)).max())}
    for name, h in (("gl2", 2.5 * dt), ("gl3", 5 * dt)):
        n = int(round(T / h))
        y = y0.clone()
        sweeps, tt, mm = 0, [], []
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(n):
            _, sw = R.step_tableau(y, k * h, h, name, tol=1e-8, max_iter=100)
            sweeps += sw
            tt.append((k + 1) * h)
            mm.append(R.dipole(y)[2].real)
        te = time.perf_counter() - ts
        res[f"{name} h={h}"] = {"rhs": n * (1 + sweeps / n * (2 if name == "gl2" else 3)), "wall_s": te,
                               "accepted": n, "rejected": 0, "mean_sweeps": sweeps / n,
                               "dipole_max_abs_vs_ref": float(np.abs(np.array(mm) - ref(np.array(tt))).max())}
        log(f"[bench] {name}: {res[f'{name} h={h}']}")
    R.close()
    base = res[f"rk4 h={dt}"]["rhs"]
    for r in res.values():
        r["rhs_ratio_rk4_over_this"] = base / r["rhs"]
    line = {
        "metric": f"right-hand sides per propagation to t={T} au by integrator (o={o} v={v}, split-BF16)",
        "value": res[f"cashkarp eps={eps:g}"]["rhs_ratio_rk4_over_this"], "unit": "RK4 RHS / Cash-Karp RHS",
        "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": f"rt-ccsd four-water-shaped synthetic o={o} v={v} seed 0, delta kick 1e-3 z, "
                               f"RK4 h={dt}, Cash-Karp and Fehlberg eps={eps:g} and {eps / 100:g}, Gauss-Legendre 2 / 3 stages at "
                               f"h={2.5 * dt} / {5 * dt} (stage sweeps to 1e-8), reference RK4 h={dt / 2}",
                   "parallelism": "single GPU"},
        "integrators": res, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_profile(args):
    """Only the RK4 steps of one precision at (o, v), from a random non-stationary state (no ground state,
    no kick, no oracle): the command to run under rocprofv3 so that its kernel summary holds the step's
    kernels alone."""
    import torch
    from paper_2205_05175_amd import RTCC
    from synth import make_system, pack_state, random_state
    o, v = args.o, args.v
    prec = args.precisions.split(",")[0]
    R = RTCC(*make_system(o, v, 0), o, v, precision="fp32" if prec == "fp64" else prec)
    R.set_precision(prec)
    y = torch.tensor(pack_state(*random_state(o, v, 3, 0.01, 0.002)), device="cuda")
    m = torch.zeros((args.warmup + args.steps + 2, 6), dtype=torch.float64, device="cuda")
    R.propagate_rk4(y, 0.0, args.dt, args.warmup, None, m[:args.warmup + 1])
    torch.cuda.synchronize()
    ts = time.perf_counter()
    R.propagate_rk4(y, args.warmup * args.dt, args.dt, args.steps, None, m[args.warmup:args.warmup + args.steps + 1])
    torch.cuda.synchronize()
    te = time.perf_counter()
    # one plain device copy of the state (2 * 16 * state entries bytes moved): the reference that scales
    # the HBM traffic counters of the step's kernels
    y.clone()
    torch.cuda.synchronize()
    log(f"[bench] profile workload {prec} o={o} v={v}: {args.steps} RK4 steps in {te - ts:.3f} s "
        f"({args.steps / (te - ts):.2f} steps/s), non-finite entries {R.check_state(y)}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["single", "spectrum", "sp-spectra", "integrators", "batch", "adjoint",
                                           "profile"],
                    default="single",
                    help="single: the o=20 v=76 propagation (default); spectrum: RK4 and Cash-Karp to t=100 au "
                         "with peak shifts; batch: 24 batched propagations; adjoint: pulse-parameter gradient at (10,38)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--gate-steps", type=int, default=500,
                    help="RK4 steps from the kick over which every precision's dipole is compared with FP64")
    ap.add_argument("--o", type=int, default=20)
    ap.add_argument("--v", type=int, default=76)
    ap.add_argument("--dt", type=float, default=0.02)
    ap.add_argument("--t-end", type=float, default=100.0, help="spectrum workload: propagation length (au)")
    ap.add_argument("--eps", type=float, default=1e-6, help="spectrum workload: Cash-Karp tolerance")
    ap.add_argument("--eps-sweep", default="", help="spectrum workload: further Cash-Karp tolerances, split-BF16 only "
                                                    "(comma-separated)")
    ap.add_argument("--sizes", default="5x19,10x38", help="sp-spectra workload: synthetic sizes oxv")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3",
                    help="single workload: the precisions to run (profiling one at a time); the JSON line needs all three")
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
    if args.workload == "integrators":
        if "--t-end" not in sys.argv:
            args.t_end = 20.0
        return bench_integrators(args)
    if args.workload == "sp-spectra":
        if "--dt" not in sys.argv:
            args.dt = 0.01
        if "--t-end" not in sys.argv:
            args.t_end = 300.0
        return bench_sp_spectra(args)
    if args.workload == "spectrum":
        return bench_spectrum(args)
    if args.workload == "profile":
        if args.steps is None:
            args.steps = 3
        return bench_profile(args)
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
    R.set_precision("fp64")
    e_corr = R.ground_state(y0, 1e-10, 200)
    torch.cuda.synchronize()
    log(f"[bench] ground state e_corr={e_corr:.12f} in {time.time() - t0:.1f} s")
    R.kick(y0, 1e-3, [0.0, 0.0, 1.0])

    W, K = args.warmup, args.steps
    G = max(args.gate_steps, W + K)
    results, traj, finals = {}, {}, {}
    precs = args.precisions.split(",")
    for prec in precs:
        R.set_precision(prec)
        y = y0.clone()
        m = torch.zeros((G + 1, 6), dtype=torch.float64, device="cuda")
        # warm-up builds the captured step graph before the timed region
        R.propagate_rk4(y, 0.0, args.dt, W, None, m[:W + 1])
        torch.cuda.synchronize()
        ts = time.perf_counter()
        R.propagate_rk4(y, W * args.dt, args.dt, K, None, m[W:W + K + 1])
        torch.cuda.synchronize()
        te = time.perf_counter()
        # kernel timing: the same steps again with HIP events around every launch of the timed class
        # (events cannot be timed inside a captured graph, so these passes issue plain launches): the
        # large complex x complex products (the dominant kernel), then the ladder GEMMs
        prof = {}
        for target in ("complex", "ladder"):
            yp = y.clone()
            mu_p = torch.zeros((K + 1, 6), dtype=torch.float64, device="cuda")
            R.profile(True, target)
            tp0 = time.perf_counter()
            R.propagate_rk4(yp, (W + K) * args.dt, args.dt, K, None, mu_p)
            prof[target] = R.profile_read()
            tp1 = time.perf_counter()
            R.profile(False)
            del yp, mu_p
        # the rest of the gate trajectory (untimed)
        if G > W + K:
            _propagate_chunked(R, y, (W + K) * args.dt, args.dt, G - W - K, m, W + K, 250, f"gate {prec}")
        bad = R.check_state(y)
        if bad:
            raise SystemExit(f"non-finite state after {prec} propagation ({bad} entries)")
        n, ms, fl, _ = prof["ladder"]
        avg = ms / max(n, 1)
        nc, msc, flc, byc = prof["complex"]
        avgc = msc / max(nc, 1)
        results[prec] = {"ms_per_step": 1e3 * (te - ts) / K, "steps_per_s": K / (te - ts),
                         "eager_ms_per_step": 1e3 * (tp1 - tp0) / K,
                         "ladder_launches": n, "ladder_ms": avg, "ladder_flops": fl,
                         "ladder_tflops": fl / (avg * 1e-3) / 1e12 if n else 0.0,
                         "cc_launches": nc, "cc_ms": avgc, "cc_flops": flc, "cc_bytes": byc,
                         "cc_tflops": flc / (avgc * 1e-3) / 1e12 if nc else 0.0}
        mm = m.cpu().numpy()
        traj[prec] = mm[:, 0::2] + 1j * mm[:, 1::2]
        finals[prec] = y
        log(f"[bench] {prec}: {results[prec]}")

    if set(precs) != {"fp64", "fp32", "bf16x3"}:
        log("[bench] not all precisions ran: no JSON line")
        return
    fp32_err = float(np.abs(traj["fp32"] - traj["fp64"]).max())
    bf16_err = float(np.abs(traj["bf16x3"] - traj["fp64"]).max())
    y64 = finals["fp64"]
    gpu_dip = R.dipole(y64)
    cpu, oracle_err = (None, None) if args.no_cpu else cpu_baseline_leg(fock, mu, o, v, y64.cpu().numpy(), gpu_dip)

    # measured ceilings of this device, reported beside the published ones (the roofline `peak`)
    from paper_2205_05175_amd import peak_probe
    measured = {"bf16_tflops": peak_probe("bf16", 6000), "fp32_tflops": peak_probe("fp32", 3000),
                "fp64_tflops": peak_probe("fp64", 3000), "hbm_copy_gbs": peak_probe("copy", 1 << 32)}
    log(f"[bench] measured peaks {measured}")
    r32 = results["fp32"]
    rbf = results["bf16x3"]
    # the headline path is split-BF16 when its dipole stays within 1e-6 au of FP64 over the gate trajectory,
    # else complex FP32
    head = "bf16x3" if bf16_err <= 1e-6 else "fp32"
    rh = results[head]
    full_ladder = os.environ.get("RTCC_LADDER", "symmetric") == "full"
    measured_traffic = head == "bf16x3" and (o, v) == (20, 76) and os.environ.get("RTCC_LADDER", "symmetric") in (
        "full", "symmetric")
    lt = LADDER_TRAFFIC_BF16X3 if full_ladder else LADDER_TRAFFIC_BF16X3_SYM
    # algorithmic minimum per launch: the packed operands read once and the complex FP32 output written
    # once (rows padded to 128, K to 32, B rows to 256; hi and lo planes of bf16)
    def packed(rows, cols, k, planes_a):
        pad = lambda x, m: -(-x // m) * m
        return (2 * pad(rows, 128) * pad(k, 32) * 2 * planes_a + 2 * pad(cols, 256) * pad(k, 32) * 2
                + rows * cols * 8)
    alg_min = (packed(2 * o * o, v * v, v * v, 2) if full_ladder else
               packed(o * (o + 1), v * (v + 1) // 2, v * (v + 1) // 2, 2)
               + packed(o * (o - 1), v * (v - 1) // 2, v * (v - 1) // 2, 2))
    peak = PEAK_TFLOPS["fp32"] if head == "fp32" else PEAK_TFLOPS["bf16"] / 3
    peak_meas = measured["fp32_tflops"] if head == "fp32" else measured["bf16_tflops"] / 3
    peak_note = ("fp32 MFMA peak" if head == "fp32" else "bf16 dense MFMA peak / 3 products per real multiply "
                 "(algorithmic fp32-equivalent flops)")
    cc_traffic = CC_TRAFFIC_BF16X3 if (measured_traffic and CC_TRAFFIC_BF16X3 and not full_ladder) else None
    sub = lambda p, key: {"achieved": results[p][key + "_tflops"], "peak": PEAK_TFLOPS[p],
                          "frac": results[p][key + "_tflops"] / PEAK_TFLOPS[p], "avg_ms": results[p][key + "_ms"],
                          "frac_of_measured": results[p][key + "_tflops"] / measured[p + "_tflops"]}
    line = {
        "metric": "RK4 steps/s (T+Λ RHS) o=20,v=76: FP32-MFMA vs FP64, dipole err vs oracle",
        "value": rh["steps_per_s"], "unit": "RK4 steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": rh["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3" if head == "bf16x3" else "f32", "data": "synthetic",
        "config": {"workload": f"rt-ccsd four-water-shaped synthetic o={o} v={v} seed 0 (factor width 0.05*24/n), "
                               f"delta kick 1e-3 z, RK4 dt={args.dt}", "o": o, "v": v,
                   "precision": ("split-bf16 three-term products (complex, fp32 accumulate) on products above "
                                 "5e8 flop, fp32 elsewhere, fp64 state" if head == "bf16x3" else
                                 "complex fp32 contractions, fp64 state"), "parallelism": "single GPU",
                   "ladder": "full o^2 v^4 product" if full_ladder else
                             "symmetric/antisymmetric pair-triangle products (a quarter of the flops)"},
        "headline_path": head,
        "gate": {"steps": G, "t_au": G * args.dt, "bound_au": 1e-6,
                 "dipole_bf16x3_vs_fp64_max_abs": bf16_err, "dipole_fp32_vs_fp64_max_abs": fp32_err},
        "fp64_steps_per_s": results["fp64"]["steps_per_s"],
        "fp32_steps_per_s": r32["steps_per_s"],
        "bf16x3_steps_per_s": rbf["steps_per_s"],
        "fp32_over_fp64": r32["steps_per_s"] / results["fp64"]["steps_per_s"],
        "bf16x3_over_fp64": rbf["steps_per_s"] / results["fp64"]["steps_per_s"],
        "dipole_fp64_gpu_vs_oracle_max_abs": oracle_err,
        # the dominant kernel: the large complex x complex products (ring and Lambda terms), 28% of the
        # split-BF16 step's kernel time at (20,76); the ladder, dominant before its symmetric form, follows
        "roofline": {"bound": "mfma",
                     "kernel": ("complex x complex split-BF16 GEMM gemm_bf16x3_nt<1, 1, 0, 4> (ring and Lambda "
                                "products; all its launches in a step)" if head == "bf16x3" else
                                "complex x complex FP32 tile GEMMs with 2 M N K >= 5e8 (ring and Lambda products)"),
                     "achieved": rh["cc_tflops"], "peak": peak, "unit": "TFLOP/s", "frac": rh["cc_tflops"] / peak,
                     "peak_note": peak_note, "peak_measured": peak_meas,
                     "frac_of_measured": rh["cc_tflops"] / peak_meas,
                     "traffic": (cc_traffic["fetch_bytes"] + cc_traffic["write_bytes"]) if cc_traffic else None,
                     "traffic_unit": "bytes per launch, mean over the step's launches (HBM, rocprofv3 FETCH_SIZE + "
                                     "WRITE_SIZE, copy-calibrated)",
                     "traffic_algorithmic_min": rh["cc_bytes"],
                     "avg_ms": rh["cc_ms"], "flops_per_launch": rh["cc_flops"],
                     "launches_per_step": rh["cc_launches"] / K,
                     "fp32": sub("fp32", "cc"), "fp64": sub("fp64", "cc")},
        "ladder_roofline": {"bound": "mfma", "kernel": (f"ladder GEMM ({head})" if full_ladder else
                                                        f"ladder GEMMs X+V+ and X-V- ({head})"),
                            "achieved": rh["ladder_tflops"],
                            "peak": peak, "unit": "TFLOP/s", "frac": rh["ladder_tflops"] / peak,
                            "peak_note": peak_note, "peak_measured": peak_meas,
                            "frac_of_measured": rh["ladder_tflops"] / peak_meas,
                            "traffic": (lt["fetch_bytes"] + lt["write_bytes"] if measured_traffic else None),
                            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                            "copy-calibrated; symmetric form: its two GEMMs in one launch)",
                            "traffic_algorithmic_min": alg_min if measured_traffic else None,
                            "avg_ms": rh["ladder_ms"], "flops_per_launch": rh["ladder_flops"],
                            "fp32": sub("fp32", "ladder"), "fp64": sub("fp64", "ladder")},
        "peak_measured": dict(measured, note="rtcc_peak_probe on this device: sustained MFMA loops (no memory "
                              "traffic) and a 4 GiB device copy (bytes read + written)"),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
