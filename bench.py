"""Benchmark of the SIPG-DG hp-multigrid hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 3D Poisson
-Laplace(u) = f on the unit cube, SIPG Q4 on 32^3 hexahedra (4,096,000
DoFs), manufactured u = prod sin(pi x_i), penalty 2(p+1)^2/h, hp V(2,2)
cycle Q4 -> Q2 -> Q1(32^3) -> 16^3 -> 8^3 -> 4^3 (dense coarsest solve).

One step = the whole hot path once, with inputs resident in HBM:
  * S fused single-touch smoother sweeps with FP64, FP32, FP16 and BF16
    storage (the 16-bit ones compute in FP32), one launch each, queued back to
    back between two HIP events on the launch stream (mean launch duration =
    elapsed / S);
  * solves to a 1e-10 relative residual from u = 0: FP64 flexible CG with the
    FP64 V-cycle, with the FP32 V-cycle (mixed precision), with the FP32
    V-cycle on 16-bit finest-level storage (FP16, BF16), and (constant kappa)
    the batched solver on this one problem (captured iteration graph).
value = FP64 fused-sweep DoF/s = DoFs / mean sweep launch duration.
Prints one JSON line (rank 0; the library runs on one GPU only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "smoother DoFs/s & time-to-1e-10 residual, mixed vs FP64 on 1 MI355X"
HBM_PEAK_GBS = 8000.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_q4_32cube_hbm_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2510_00998_amd", "csrc", "dg_kernels_impl.hpp")


def counter_traffic(key):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILE).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        line = line.strip()
        if ":" in line and (line.startswith("source_sha256") or line.startswith("traffic_bytes")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != sha or key not in vals:
        return None
    return float(vals[key])


def measured_copy_bandwidth(torch, dev, stream, mib=1024, reps=10):
    """Read + write bytes per second of a plain device-to-device copy of
    `mib` MiB (the achievable streaming rate, beside the datasheet peak)."""
    a = torch.empty(mib * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        c.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, c
    return 2 * mib * 1024 * 1024 / t / 1e9


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=20, help="fused sweeps per precision per step")
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5],
                    help="2: Q4 32^3 kappa=1 (headline); 3: Q3 64^3 log-uniform kappa; "
                         "4: 64 problems x 4 RHS batched; 5: Q5 96^3 log-normal kappa")
    ap.add_argument("--paper-tables", action="store_true",
                    help="paper-mode cycle counts: 2D, one-step DG_p -> Q1, factor-3 h-coarsening, MGMult to 1e-7")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=6, help="mesh of the oracle's timed sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of known size (for counter calibration)")
    return ap.parse_args()


def cpu_baseline(dim, p, n_sample):
    """The oracle (assembled CSR block-Jacobi and MG-PCG, FP64) timed on a
    bounded sample of the same workload (same dim, p, kappa, f; smaller mesh)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import Hierarchy, manufactured as mf

    with threadpool_limits(limits=1):
        H = Hierarchy(dim, n_sample, p)
        _, f = mf.sin_product(dim, 1)
        b = H.fine.load_vector(f)
        u = np.zeros_like(b)
        nd = H.fine.ndof
        sweeps, t = 0, 0.0
        t0 = time.perf_counter()
        while t < 8.0 or sweeps < 2:
            u = H.smooth(0, u, b, 1)
            sweeps += 1
            t = time.perf_counter() - t0
        sweep_rate = nd * sweeps / t
        t0 = time.perf_counter()
        _, hist = H.solve(b, rtol=1e-10, maxit=200)
        tsolve = time.perf_counter() - t0
    return {
        "value": sweep_rate, "unit": "DoF/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle block-Jacobi sweeps (assembled CSR matvec + dense Cholesky blocks), "
                   f"{dim}D Q{p} on {n_sample}^{dim} cells ({nd} DoFs), {sweeps} sweeps in {t:.1f} s; "
                   f"oracle MG-PCG to 1e-10 on the same mesh: {len(hist) - 1} its in {tsolve:.1f} s"),
        "time_to_1e-10_s_sample": tsolve,
    }


def run_batched(args):
    """64 independent 3D Poisson problems (n uniform in 8..48, p uniform in
    1..5, seed 1004), 4 right-hand sides N(0,1) per DoF each, solved together
    by the batched solver.  One step = batched FP64 and FP32 smoothing of all
    problems (S sweeps each) + one batched mixed-precision solve to 1e-10.
    Afterwards, once: the same problems solved one after another by the
    single-problem solver with the FP32 cycle and with the FP64 cycle."""
    import torch

    import paper_2510_00998_amd as hp
    import synth
    from paper_2510_00998_amd import traffic

    probs = synth.batched_problem_list()
    R = 4
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t_setup = time.perf_counter()
    solvers = [hp.Solver(3, n, p, 1.0, max_rhs=R, precision=hp.PREC_F32) for n, p in probs]
    batch = hp.Batch(solvers)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    _progress(f"set up {len(solvers)} problems in {t_setup:.1f} s")
    ndofs = [s.ndof for s in solvers]
    total = R * sum(ndofs)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1004)
    bs = [torch.randn(R * nd, dtype=torch.float64, device=dev, generator=gen) for nd in ndofs]
    us = [torch.zeros_like(b) for b in bs]
    bs32 = [b.float() for b in bs]
    us32 = [torch.zeros_like(b) for b in bs32]
    S = args.sweeps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    # first calls build the tables and tune the persistent grids (untimed)
    batch.smooth(us, bs, 0, nrhs=R)
    batch.smooth(us32, bs32, 0, nrhs=R)
    torch.cuda.synchronize()

    def step(record):
        out = {}
        for k, (uu, bb) in enumerate(((us, bs), (us32, bs32))):
            e = evs[3 * k:3 * k + 3]
            e[0].record(stream)
            batch.smooth(uu, bb, 0, nrhs=R)
            e[1].record(stream)
            batch.smooth(uu, bb, S, nrhs=R)
            e[2].record(stream)
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, st = batch.solve(us, bs, rtol=1e-10, maxit=200, nrhs=R)
        out["solve"] = (time.perf_counter() - t0, max(i.iterations for i in infos), st)
        if record:
            for k, name in ((0, "f64"), (1, "f32")):
                e = evs[3 * k:3 * k + 3]
                tp = e[0].elapsed_time(e[1]) * 1e-3
                ts = e[1].elapsed_time(e[2]) * 1e-3
                out[name] = (ts - tp) / S
        return out

    for i in range(args.warmup):
        step(False)
        _progress(f"warm-up step {i} done")
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    res = []
    for i in range(args.steps):
        res.append(step(True))
        _progress(f"step {i}: batched solve {res[-1]['solve'][0]:.3f} s, {res[-1]['solve'][1]} its")
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    t64 = sum(r["f64"] for r in res) / len(res)
    t32 = sum(r["f32"] for r in res) / len(res)
    t_batch = min(r["solve"][0] for r in res)
    its_batch = res[-1]["solve"][1]
    ok = all(r["solve"][2] == 0 for r in res)

    # worst true relative residual of the batched solutions (FP64 apply)
    worst = 0.0
    for s, u, b in zip(solvers, us, bs):
        y = torch.empty_like(u)
        s.apply_A(u, y, nrhs=R)
        for r in range(R):
            sl = slice(r * s.ndof, (r + 1) * s.ndof)
            worst = max(worst, float(torch.linalg.vector_norm(b[sl] - y[sl]) / torch.linalg.vector_norm(b[sl])))

    # the same problems one after another: single-problem solver, FP32 cycle
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_seq_mx = 0
    for s, u, b in zip(solvers, us, bs):
        u.zero_()
        info, st = s.solve(u, b, rtol=1e-10, maxit=200, nrhs=R)
        its_seq_mx = max(its_seq_mx, info.iterations)
        ok = ok and st == 0
    torch.cuda.synchronize()
    t_seq_mx = time.perf_counter() - t0
    _progress(f"sequential mixed solves {t_seq_mx:.3f} s")
    tuning = batch.tuning
    by64 = R * sum(traffic.sweep_bytes(3, n, p, 8) for n, p in probs)
    by32 = R * sum(traffic.sweep_bytes(3, n, p, 4) for n, p in probs)
    del us32, bs32, batch
    del solvers
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # FP64 cycle, one problem after another (set up one at a time)
    t_seq_64 = 0.0
    its_seq_64 = 0
    for (n, p), u, b in zip(probs, us, bs):
        s = hp.Solver(3, n, p, 1.0, max_rhs=R, precision=hp.PREC_F64)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, st = s.solve(u, b, rtol=1e-10, maxit=200, nrhs=R)
        torch.cuda.synchronize()
        t_seq_64 += time.perf_counter() - t0
        its_seq_64 = max(its_seq_64, info.iterations)
        ok = ok and st == 0
        s.close()
    _progress(f"sequential FP64 solves {t_seq_64:.3f} s")

    ach = by64 / t64 / 1e9
    line = {
        "metric": METRIC,
        "value": total / t64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "64 independent 3D Poisson SIPG problems, n uniform in 8..48, p uniform in 1..5 "
                               "(seed 1004), 4 RHS N(0,1) per DoF each, batched: one launch per phase over all "
                               "problems, captured FCG iteration, FP32 V(2,2) inside FP64 FCG to 1e-10",
                   "problems": len(probs), "rhs": R, "total_dofs": total, "sweeps_per_step": S},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_dg_batch<double,BOP_SWEEP> (batched fused sweep of all problems, FP64)",
                     "algorithmic_bytes_per_launch": by64, "mean_launch_s": t64},
        "sweep_dofs_per_s": {"f64": total / t64, "f32": total / t32},
        "sweep_roofline_f32": {"achieved": by32 / t32 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": by32 / t32 / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": by32,
                               "mean_launch_s": t32},
        "time_to_1e-10_s": {"batched_mixed": t_batch, "sequential_mixed": t_seq_mx, "sequential_fp64": t_seq_64},
        "solver_iterations": {"batched_mixed": its_batch, "sequential_mixed": its_seq_mx,
                              "sequential_fp64": its_seq_64},
        "solves_converged": ok,
        "batched_worst_true_rel_residual": worst,
        "autotuned_launch": tuning,
        "setup_s": t_setup,
    }
    print(json.dumps(line), flush=True)


def run_paper_tables(args):
    """Cycles of the stationary multigrid iteration (MGMult, FP64) to reduce the
    unpreconditioned or the preconditioned relative residual by 1e-7, in the
    paper's 2D setting: unit square, n^2 cells (n = 9 .. 243), p = 2 .. 6,
    one-step p-coarsening DG_p -> Q1, factor-3 h-coarsening to 3^2, V(2,2),
    for the sin-product and the two-peak manufactured solutions."""
    import torch

    import paper_2510_00998_amd as hp

    meshes = (9, 27, 81, 243)
    degrees = (2, 3, 4, 5, 6)
    bases = ("gll", "gl")
    counts = {bs: {e: {s: {} for s in ("sin_product", "two_peak")} for e in ("unprec", "prec")} for bs in bases}
    secs = {bs: {e: {s: {} for s in ("sin_product", "two_peak")} for e in ("unprec", "prec")} for bs in bases}
    T0 = time.perf_counter()
    for bi, bs in enumerate(bases):
        for sol, kind in (("sin_product", 1), ("two_peak", 2)):
            for n in meshes:
                for p in degrees:
                    g = hp.Solver(2, n, p, 1.0, p_coarsening=1, h_factor=3, coarsest_n=3, precision=hp.PREC_F64,
                                  basis=bi)
                    b = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
                    g.load_vector(kind, 2.0, b)
                    for ex in ("unprec", "prec"):
                        u = torch.zeros_like(b)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        info, st = g.mgmult(u, b, rtol=1e-7, maxit=1000, exit=ex, check=False)
                        torch.cuda.synchronize()
                        counts[bs][ex][sol].setdefault(f"{n}x{n}", {})[p] = info.iterations if st == 0 else None
                        secs[bs][ex][sol].setdefault(f"{n}x{n}", {})[p] = time.perf_counter() - t0
                    g.close()
                _progress(f"{bs} {sol} n={n} done")
    line = {
        "metric": "paper-mode hp-multigrid cycles to 1e-7 (2D)", "value": None, "unit": "cycles",
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": "2D Poisson, SIPG Q_p on n^2 cells (Gauss-Lobatto and Gauss-Legendre nodes), "
                               "manufactured sin(2 pi x)sin(2 pi y) and two-peak solutions, MGMult with V(2,2) "
                               "(omega_DG 0.7, omega_CG 2/3), one-step DG_p -> Q1, factor-3 h-coarsening to 3^2, FP64",
                   "meshes": list(meshes), "degrees": list(degrees)},
        "cycles": counts, "seconds": secs, "total_s": time.perf_counter() - T0,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on exactly one GPU; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    if args.paper_tables:
        run_paper_tables(args)
        return
    if args.config == 4:
        run_batched(args)
        return
    import torch

    import paper_2510_00998_amd as hp
    from paper_2510_00998_amd import traffic

    import synth
    dim = 3
    if args.config == 2:
        n, p, kappa, fkind, wl = 32, 4, 1.0, 1, "u=prod sin(pi x_i)"
    elif args.config == 3:
        n, p, fkind = 64, 3, 0
        kappa = synth.kappa_log_uniform(3, n, seed=1003)
        wl = "kappa log-uniform in [1e-2,1e2] per cell (seed 1003), f=1"
    else:
        n, p, fkind = 96, 5, 0
        kappa = synth.kappa_log_normal(3, n, seed=1005)
        wl = "kappa log-normal (sigma_log 2, correlation length 0.1, seed 1005), f=1"
    vark = not isinstance(kappa, float)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t_setup = time.perf_counter()
    g64 = hp.Solver(dim, n, p, kappa, precision=hp.PREC_F64)
    gmx = hp.Solver(dim, n, p, kappa, precision=hp.PREC_F32)
    g16 = hp.Solver(dim, n, p, kappa, precision=hp.PREC_F16)
    gb16 = hp.Solver(dim, n, p, kappa, precision=hp.PREC_BF16)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    nd = g64.ndof
    b64 = torch.empty(nd, dtype=torch.float64, device=dev)
    g64.load_vector(fkind, 1.0, b64)
    # sweep inputs per storage type; 16-bit b scaled to mean square
    # lambda = d pi^2 kappa_min (h/N)^d like the solver's 16-bit cycles, so
    # that the iterates stay in FP16 range
    import math
    kmin = kappa if not vark else float(min(kappa))
    lam = dim * math.pi ** 2 * kmin * (1.0 / (n * (p + 1))) ** dim
    bscale = float((nd * lam) ** 0.5 / torch.linalg.vector_norm(b64))
    sweep_in = {}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32), ("f16", torch.float16),
                     ("bf16", torch.bfloat16)):
        bb = b64 if dt == torch.float64 else (b64 * (1.0 if dt == torch.float32 else bscale)).to(dt)
        sweep_in[name] = (torch.zeros(nd, dtype=dt, device=dev), bb,
                          [torch.cuda.Event(enable_timing=True) for _ in range(2)])
    u = torch.zeros(nd, dtype=torch.float64, device=dev)
    # the same sweep with Gauss-Legendre nodes (dense facet value functionals)
    ggl = hp.Solver(dim, n, p, kappa, basis=1)
    gl_in = {name: (torch.zeros(nd, dtype=dt, device=dev), b64.to(dt),
                    [torch.cuda.Event(enable_timing=True) for _ in range(2)])
             for name, dt in (("f64", torch.float64), ("f32", torch.float32))}
    solves = ("fp64", "mixed_f32", "mixed_f16", "mixed_bf16")
    if not vark:
        solves += ("mixed_f32_graph",)
    solver_of = {"fp64": g64, "mixed_f32": gmx, "mixed_f16": g16, "mixed_bf16": gb16}
    # variable kappa: the same sweeps and mixed solve with the block inverse
    # rebuilt in every traversal from kappa (no stored per-cell eigendata)
    rc_in = {}
    t_setup_rc = None
    if vark:
        t0 = time.perf_counter()
        grc = hp.Solver(dim, n, p, kappa, block_recompute=1)
        torch.cuda.synchronize()
        t_setup_rc = time.perf_counter() - t0
        rc_in = {name: (torch.zeros(nd, dtype=dt, device=dev), b64.to(dt),
                        [torch.cuda.Event(enable_timing=True) for _ in range(2)])
                 for name, dt in (("f64", torch.float64), ("f32", torch.float32))}
        solves += ("mixed_f32_block_recompute",)
        solver_of["mixed_f32_block_recompute"] = grc
    batch1 = None if vark else hp.Batch([gmx])
    S = args.sweeps

    def step(record):
        out = {}
        # S fused sweeps (one hpmg_sweep call, one launch per sweep) queued
        # back to back between two events on the launch stream:
        # mean launch duration = elapsed / S
        for gs, ins in ((g64, sweep_in), (ggl, gl_in)) + (((grc, rc_in),) if vark else ()):
            for uu, bb, evs in ins.values():
                gs.project(uu)
                evs[0].record(stream)
                gs.sweep(uu, bb, S)
                evs[1].record(stream)
        # time to 1e-10: FP64 cycle, then mixed FP32 cycle (single-problem
        # solver; and, for constant kappa, the batched solver on a batch of
        # one, whose iteration is a captured graph)
        for name in solves:
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "mixed_f32_graph":
                infos, st = batch1.solve([u], [b64], rtol=1e-10, maxit=200)
                info = infos[0]
            else:
                info, st = solver_of[name].solve(u, b64, rtol=1e-10, maxit=200, check=False)
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0, info.iterations, st,
                         info.final_residual / max(info.initial_residual, 1e-300))
        if record:
            for name, (_, _, evs) in sweep_in.items():
                out["sw_" + name] = evs[0].elapsed_time(evs[1]) * 1e-3 / S
            for name, (_, _, evs) in gl_in.items():
                out["swgl_" + name] = evs[0].elapsed_time(evs[1]) * 1e-3 / S
            for name, (_, _, evs) in rc_in.items():
                out["swrc_" + name] = evs[0].elapsed_time(evs[1]) * 1e-3 / S
        return out

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    res = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    T = time.perf_counter() - T0

    tsw = {name: sum(r["sw_" + name] for r in res) / len(res) for name in sweep_in}
    isz = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
    bysw = {name: traffic.sweep_bytes(dim, n, p, isz[name], per_cell_kappa=vark) for name in sweep_in}
    t64, t32 = tsw["f64"], tsw["f32"]
    by64, by32 = bysw["f64"], bysw["f32"]
    tt = {k: min(r[k][0] for r in res) for k in solves}
    its = {k: res[-1][k][1] for k in solves}
    conv = {k: all(r[k][2] == 0 for r in res) for k in solves}
    final_rel = {k: res[-1][k][3] for k in solves}
    ok = all(conv[k] for k in ("fp64", "mixed_f32"))

    # true residual of the mixed-precision (FP32 cycle) solution (FP64 apply)
    u.zero_()
    gmx.solve(u, b64, rtol=1e-10, maxit=200, check=False)
    y = torch.empty_like(u)
    g64.apply_A(u, y)
    true_rel = float(torch.linalg.vector_norm(b64 - y) / torch.linalg.vector_norm(b64))

    if args.copy_calibration:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
    copy_gbs = measured_copy_bandwidth(torch, dev, stream)

    ach64 = by64 / t64 / 1e9
    headline = args.config == 2
    tkey64 = "traffic_bytes_per_launch_f64" if headline else "none"
    tkey32 = "traffic_bytes_per_launch_f32" if headline else "none"
    line = {
        "metric": METRIC,
        "value": nd / t64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D SIPG Q{p} on {n}^3 hexes ({nd} DoFs), {wl}, "
                               "fused single-touch block-Jacobi sweep + hp V(2,2) (p halved to Q1, h to <=4^3), "
                               "FCG to 1e-10",
                   "dim": dim, "n": n, "p": p, "ndof": nd, "sweeps_per_step": S},
        "roofline": {"bound": "hbm", "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach64 / HBM_PEAK_GBS, "traffic": counter_traffic(tkey64),
                     "kernel": f"k_sweep<double,3,{p + 1}> (fused sweep, FP64)",
                     "algorithmic_bytes_per_launch": by64, "mean_launch_s": t64,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": ach64 / copy_gbs},
        "sweep_dofs_per_s": {name: nd / t for name, t in tsw.items()},
        "sweep_dofs_per_s_gauss_legendre": {name: nd / (sum(r["swgl_" + name] for r in res) / len(res))
                                            for name in gl_in},
        "sweep_roofline_f32": {"achieved": by32 / t32 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": by32 / t32 / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": by32,
                               "traffic": counter_traffic(tkey32),
                               "mean_launch_s": t32},
        "sweep_roofline_16bit_storage": {
            name: {"achieved": bysw[name] / tsw[name] / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": bysw[name] / tsw[name] / 1e9 / HBM_PEAK_GBS,
                   "algorithmic_bytes_per_launch": bysw[name], "mean_launch_s": tsw[name]}
            for name in ("f16", "bf16")},
        "time_to_1e-10_s": tt,
        "solver_iterations": its,
        "solves_converged": ok,
        "converged_by_solver": conv,
        "final_rel_residual_by_solver": final_rel,
        "mixed_solution_true_rel_residual": true_rel,
        "setup_s": t_setup,
    }
    if vark:
        trc = {name: sum(r["swrc_" + name] for r in res) / len(res) for name in rc_in}
        byrc = {name: traffic.sweep_bytes(dim, n, p, isz[name], per_cell_kappa=True, block_recompute=True)
                for name in rc_in}
        line["block_recompute"] = {
            "setup_s": t_setup_rc,
            "sweep_dofs_per_s": {name: nd / t for name, t in trc.items()},
            "sweep_mean_launch_s": trc,
            "sweep_roofline_frac": {name: byrc[name] / trc[name] / 1e9 / HBM_PEAK_GBS for name in rc_in},
            "algorithmic_bytes_per_launch": byrc}
    if not args.no_cpu_baseline and headline:
        line["cpu_baseline"] = cpu_baseline(dim, p, args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
