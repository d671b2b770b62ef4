"""Benchmark of the SIPG-DG hp-multigrid hot path on one MI355X.

Default workload (the largest configuration that fits one GPU): 64
independent 3D Poisson problems, SIPG Q_p on n^3 hexahedra with n uniform in
8..48 and p uniform in 1..5 (seed 1004), 4 right-hand sides drawn N(0,1) per
DoF each (918,658,044 DoFs over all right-hand sides), solved together by
the batched driver: one persistent launch per V-cycle phase over all
problems, one FCG iteration captured as a HIP graph, FP32 V(2,2) cycle inside
the FP64 flexible CG, to a 1e-10 relative residual.

One step = the whole hot path once, inputs resident in HBM:
  * S fused single-touch block-Jacobi sweeps of every problem and right-hand
    side in FP64 and in FP32 (hpmg_batch_smooth: one projection launch, then
    per sweep one launch per polynomial degree), bracketed by HIP events on
    the launch stream: mean sweep time = (t(projection + S sweeps) -
    t(projection)) / S;
  * the batched mixed-precision solve of all 256 segments from u = 0.
After the timed steps, once (median of --seq-reps repetitions): the same
problems solved one after another by the single-problem solver with the FP32
cycle and with the FP64 cycle.

value = FP64 sweep DoF/s over all problems and right-hand sides.
--config 2|3|5 measures the single-problem workloads (Q4 32^3, Q3 64^3 with
log-uniform kappa, Q5 96^3 with log-normal kappa); --config 6 the adaptive
spacetree workload (Q4 on 16^3 base cells refined twice by 2 around two
balls, 33,734 leaves); --paper-tables the paper's 2D cycle-count study.  Prints one JSON line (the library runs on one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "smoother DoFs/s & time-to-1e-10 residual, mixed vs FP64 on 1 MI355X"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2510_00998_amd", "csrc")


def _sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def counter_traffic(summary, sources, key, require=None):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None if the kernel sources have
    changed since the counters were taken, or if a `require` entry (launch
    configuration) differs from the one recorded with the counters."""
    try:
        txt = open(os.path.join(ROOT, "profiles", summary)).read()
        sha = _sha(sources)
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        line = line.strip()
        if ":" in line and (line.startswith("source_sha256") or line.startswith("traffic_bytes")
                            or line.startswith("launch_")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != sha or key not in vals:
        return None
    for k, v in (require or {}).items():
        if vals.get(k) != v:
            return None
    return float(vals[key])


def recorded_launch(summary, sources):
    """The batched launch configuration (hpmg_batch_tuning's 9 ints) recorded
    with a committed counter profile, or None if the kernel sources have
    changed since (then the autotuner's own choice is timed)."""
    try:
        txt = open(os.path.join(ROOT, "profiles", summary)).read()
        sha = _sha(sources)
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line:
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != sha or "launch_tuning_raw" not in vals:
        return None
    return [int(x) for x in vals["launch_tuning_raw"].split(",")]


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


def copy_calibration(torch, dev):
    """Three plain device copies of 256 MiB (the counter calibration of the
    profiles: bytes read and written are known)."""
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _median(xs):
    return statistics.median(xs) if xs else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=20, help="fused sweeps per precision per step")
    ap.add_argument("--config", type=int, default=4, choices=[2, 3, 4, 5, 6],
                    help="4: 64 problems x 4 RHS batched (default, largest workload); 2: Q4 32^3 kappa=1; "
                         "3: Q3 64^3 log-uniform kappa; 5: Q5 96^3 log-normal kappa; 6: Q4 adaptive spacetree "
                         "(16^3 base cells, two levels of refinement by 2 around two balls)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="paper-mode cycle counts: 2D, one-step DG_p -> Q1, factor-3 h-coarsening, MGMult to 1e-7")
    ap.add_argument("--profile-sweeps", action="store_true",
                    help="only setup, autotuning and S timed sweeps per precision (for rocprofv3 runs)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="single-problem configs: setup, then three solves with the FP32 cycle only (for rocprofv3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="oracle sweep time (batched: per two sample problems)")
    ap.add_argument("--block-recompute", action="store_true",
                    help="with --profile-sweeps and variable kappa: time the sweeps that rebuild the block inverse "
                         "in every traversal instead of the stored-eigendata sweeps (same kernel names, so each "
                         "variant is profiled in its own process)")
    ap.add_argument("--seq-reps", type=int, default=3, help="repetitions of the problem-after-problem solves")
    ap.add_argument("--smooth-tuning", default=None,
                    help="batched workload: 9 comma-separated ints for hpmg_batch_set_tuning after the first calls "
                         "(a launch configuration recorded with a profile)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of known size (for counter calibration)")
    return ap.parse_args()


# ----------------------------------------------------------------- CPU side
def cpu_baseline_cpp(problems, seconds, label):
    """The C++ oracle (oracle/coracle.py: assembled CSR SIPG, block-Jacobi with
    dense Cholesky blocks, Galerkin V-cycle, FCG; OpenMP over all host cores
    given to it, at most 16, the GPU machine's share) on each sample problem in
    turn: block-Jacobi sweeps for about `seconds`, then one MG-PCG solve to
    1e-10.  value = DoF sweeps per second over the sample."""
    os.environ.setdefault("OMP_NUM_THREADS", str(min(16, os.cpu_count() or 1)))
    from oracle.coracle import CHierarchy, threads

    import numpy as np

    import synth

    runs = []
    for n, p, seed in problems:
        t0 = time.perf_counter()
        H = CHierarchy(3, n, p, 1.0)
        t_setup = time.perf_counter() - t0
        b = synth.random_rhs(H.ndof, seed=seed)
        u = np.zeros_like(b)
        sweeps, t = 0, 0.0
        t0 = time.perf_counter()
        while t < seconds or sweeps < 2:
            u = H.smooth(u, b, 1)
            sweeps += 1
            t = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, hist = H.solve(b, rtol=1e-10, maxit=300)
        ts = time.perf_counter() - t0
        runs.append({"n": n, "p": p, "ndof": H.ndof, "setup_s": t_setup, "sweeps": sweeps, "sweep_s": t,
                     "solve_s": ts, "its": len(hist) - 1})
    rate = sum(r["ndof"] * r["sweeps"] for r in runs) / sum(r["sweep_s"] for r in runs)
    return {
        "value": rate, "unit": "DoF/s", "cores": threads(), "kind": "oracle",
        "sample": (f"{label}: the C++ oracle with {threads()} OpenMP threads, per problem block-Jacobi sweeps "
                   f"(assembled CSR matvec + dense Cholesky blocks) for about {seconds:.0f} s, then one MG-PCG "
                   "solve to 1e-10"),
        "runs": runs,
        "time_to_1e-10_s_sample": {f"n{r['n']}_p{r['p']}": r["solve_s"] for r in runs},
    }


# --------------------------------------------------------------- batched
def run_batched(args):
    """64 independent 3D Poisson problems (n uniform in 8..48, p uniform in
    1..5, seed 1004), 4 right-hand sides N(0,1) per DoF each, solved together
    by the batched solver."""
    import synth
    probs = synth.batched_problem_list()
    R = 4
    base = None
    if not args.no_cpu_baseline and not args.profile_sweeps:
        # the oracle on the six smallest problems of the batch
        order = sorted(range(len(probs)), key=lambda j: probs[j][0] ** 3 * (probs[j][1] + 1) ** 3)[:6]
        _progress("oracle baseline on the six smallest problems")
        base = cpu_baseline_cpp([(probs[j][0], probs[j][1], synth.batched_rhs_seed(1004, j, 0)) for j in order],
                                args.cpu_seconds / 2,
                                "the six smallest problems of the batch "
                                + ", ".join(f"Q{probs[j][1]} {probs[j][0]}^3" for j in order))

    import torch

    import paper_2510_00998_amd as hp
    from paper_2510_00998_amd import traffic

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
    # the first calls build the tables and tune the persistent grids (untimed)
    batch.smooth(us, bs, 0, nrhs=R)
    batch.smooth(us32, bs32, 0, nrhs=R)
    torch.cuda.synchronize()
    autotuned = batch.tuning
    # the timed smoothing runs the launch configuration recorded with the
    # committed counter profile (so that roofline.traffic describes exactly
    # the timed kernels; the autotuner's choice among near-equal
    # configurations varies from run to run), else the autotuned one
    srcs = ["dg_kernels_impl.hpp", "batch_dg_body.hpp", "batch_kernels.hip"]
    forced = [int(x) for x in args.smooth_tuning.split(",")] if args.smooth_tuning else None
    if forced is None and not args.profile_sweeps:
        forced = recorded_launch("batched_64x4_hbm_traffic.md", srcs)
    if forced is not None:
        # smoothing parts only; the V-cycle tunes at its first solve
        batch.set_tuning([0, 0] + forced[2:6] + [0] + forced[7:9])
    tuning = batch.tuning
    raw = batch.tuning_raw
    # smoothing launch configuration as recorded with the counter profile:
    # one launch per degree or one for all, and the half-tile degree mask
    launch_cfg = {"launch_smooth_f64": f"split={raw[5]} tile={raw[8]}",
                  "launch_smooth_f32": f"split={raw[3]} tile={raw[7]}"}

    def smooth_timed():
        out = {}
        for k, (name, uu, bb) in enumerate((("f64", us, bs), ("f32", us32, bs32))):
            e = evs[3 * k:3 * k + 3]
            e[0].record(stream)
            batch.smooth(uu, bb, 0, nrhs=R)
            e[1].record(stream)
            batch.smooth(uu, bb, S, nrhs=R)
            e[2].record(stream)
        torch.cuda.synchronize()
        for k, name in ((0, "f64"), (1, "f32")):
            e = evs[3 * k:3 * k + 3]
            out[name] = (e[1].elapsed_time(e[2]) - e[0].elapsed_time(e[1])) * 1e-3 / S
        return out

    by64 = R * sum(traffic.sweep_bytes(3, n, p, 8) for n, p in probs)
    by32 = R * sum(traffic.sweep_bytes(3, n, p, 4) for n, p in probs)
    degs = sorted({p for _, p in probs})
    if args.profile_sweeps:
        t = smooth_timed()
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"profile_sweeps": S, "mean_sweep_s": t, "algorithmic_bytes": {"f64": by64, "f32": by32},
                          "autotuned_launch": autotuned,
        "timed_launch": tuning,
        "timed_launch_source": ("--smooth-tuning" if args.smooth_tuning else
                                "recorded with profiles/batched_64x4_hbm_traffic.md" if forced else "autotuned"), "tuning_raw": raw, "launch_config": launch_cfg}), flush=True)
        return

    def step():
        out = smooth_timed()
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, st = batch.solve(us, bs, rtol=1e-10, maxit=200, nrhs=R, check=False)
        out["solve"] = (time.perf_counter() - t0, max(i.iterations for i in infos), st)
        return out

    for i in range(args.warmup):
        step()
        _progress(f"warm-up step {i} done")
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    res = []
    for i in range(args.steps):
        res.append(step())
        _progress(f"step {i}: batched solve {res[-1]['solve'][0]:.3f} s, {res[-1]['solve'][1]} its")
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    t64 = _median([r["f64"] for r in res])
    t32 = _median([r["f32"] for r in res])
    ok_batch = all(r["solve"][2] == 0 for r in res)
    t_batch = _median([r["solve"][0] for r in res]) if ok_batch else None
    its_batch = res[-1]["solve"][1]

    # worst true relative residual of the batched solutions (FP64 apply)
    worst = 0.0
    for s, u, b in zip(solvers, us, bs):
        y = torch.empty_like(u)
        s.apply_A(u, y, nrhs=R)
        for r in range(R):
            sl = slice(r * s.ndof, (r + 1) * s.ndof)
            worst = max(worst, float(torch.linalg.vector_norm(b[sl] - y[sl]) / torch.linalg.vector_norm(b[sl])))

    # the same problems one after another: single-problem solver, FP32 cycle
    seq_mx, its_seq_mx, ok_mx = [], 0, True
    for rep in range(args.seq_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, u, b in zip(solvers, us, bs):
            u.zero_()
            info, st = s.solve(u, b, rtol=1e-10, maxit=200, nrhs=R, check=False)
            its_seq_mx = max(its_seq_mx, info.iterations)
            ok_mx = ok_mx and st == 0
        torch.cuda.synchronize()
        seq_mx.append(time.perf_counter() - t0)
    _progress(f"problem after problem, FP32 cycle: {seq_mx}")
    del us32, bs32, batch
    del solvers
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # FP64 cycle, one problem after another (set up one at a time); per
    # problem the median of the repetitions, summed
    seq_64, its_seq_64, ok_64 = 0.0, 0, True
    for (n, p), u, b in zip(probs, us, bs):
        s = hp.Solver(3, n, p, 1.0, max_rhs=R, precision=hp.PREC_F64)
        ts = []
        for rep in range(args.seq_reps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info, st = s.solve(u, b, rtol=1e-10, maxit=200, nrhs=R, check=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            its_seq_64 = max(its_seq_64, info.iterations)
            ok_64 = ok_64 and st == 0
        seq_64 += statistics.median(ts)
        s.close()
    _progress(f"problem after problem, FP64 cycle: {seq_64:.3f} s")

    copy_gbs = measured_copy_bandwidth(torch, dev, stream)
    ach = by64 / t64 / 1e9
    split = tuning["smooth_f64_split_by_degree"]
    half = set(tuning["smooth_f64_half_tile_degrees"])
    one = "true" if tuning["smooth_f64_grid"] > 8192 else "false"  # the grid covers the item list
    kern64 = (f"k_dg_batch_n<double,0,N,V,{one}> for (N,V) = " +
              ",".join(f"({p + 1},{int(p in half)})" for p in degs) +
              " (one launch per degree per sweep; V = 1: half the cells per workgroup; true: one workgroup per"
              " work item)") if split \
        else "k_dg_batch<double,0> (one launch per sweep)"
    # time-to-solution roofline: bytes of one FCG iteration of every segment
    # (the captured graph iterates all segments until the last converges)
    iter_bytes = R * sum(traffic.fcg_iteration_bytes(3, n, p, 4) for n, p in probs)
    tts = None
    if t_batch:
        a = iter_bytes * its_batch / t_batch / 1e9
        tts = {"achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
               "bytes_per_iteration": iter_bytes, "iterations": its_batch, "seconds": t_batch}
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
                               "(seed 1004), 4 RHS N(0,1) per DoF each (918,658,044 DoFs), batched: one launch per "
                               "phase over all problems, captured FCG iteration, FP32 V(2,2) inside FP64 FCG to 1e-10",
                   "problems": len(probs), "rhs": R, "total_dofs": total, "sweeps_per_step": S},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": counter_traffic("batched_64x4_hbm_traffic.md", srcs, "traffic_bytes_per_sweep_f64",
                                                {"launch_smooth_f64": launch_cfg["launch_smooth_f64"]}),
                     "kernel": kern64 + " (batched fused sweep of all problems and RHS, FP64)",
                     "algorithmic_bytes_per_launch": by64, "mean_launch_s": t64,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": ach / copy_gbs},
        "sweep_dofs_per_s": {"f64": total / t64, "f32": total / t32},
        "sweep_roofline_f32": {"achieved": by32 / t32 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": by32 / t32 / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": by32,
                               "traffic": counter_traffic("batched_64x4_hbm_traffic.md", srcs,
                                                          "traffic_bytes_per_sweep_f32",
                                                          {"launch_smooth_f32": launch_cfg["launch_smooth_f32"]}),
                               "mean_launch_s": t32},
        "time_to_1e-10_s": {"batched_mixed": t_batch, "sequential_mixed": _median(seq_mx) if ok_mx else None,
                            "sequential_fp64": seq_64 if ok_64 else None},
        "time_to_solution_roofline_batched": tts,
        "solver_iterations": {"batched_mixed": its_batch, "sequential_mixed": its_seq_mx,
                              "sequential_fp64": its_seq_64},
        "solves_converged": {"batched_mixed": ok_batch, "sequential_mixed": ok_mx, "sequential_fp64": ok_64},
        "batched_worst_true_rel_residual": worst,
        "autotuned_launch": autotuned,
        "timed_launch": tuning,
        "timed_launch_source": ("--smooth-tuning" if args.smooth_tuning else
                                "recorded with profiles/batched_64x4_hbm_traffic.md" if forced else "autotuned"),
        "setup_s": t_setup,
    }
    if base is not None:
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


# ----------------------------------------------------------- paper tables
def run_paper_tables(args):
    """Cycles of the stationary multigrid iteration (Algorithm MGMult, FP64) to
    reduce the unpreconditioned or the preconditioned relative residual by
    1e-7 in the paper's 2D setting: unit square, n^2 cells (n = 9 .. 243),
    p = 2 .. 6, one-step p-coarsening DG_p -> Q1, factor-3 h-coarsening to
    3^2, nu block-Jacobi pre- and zero post-smoothing steps with the
    interior-cell block on the DG level, for the sin-product and the
    two-peak manufactured solutions, over a scan of the parameters the paper
    does not print (nu, omega_DG, the penalty factor sigma0, the Q1 smoothing
    counts); the distance to the paper's counts is reported per setting."""
    import math

    import torch

    import paper_2510_00998_amd as hp

    paper = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_cycle_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        ex, sol, n, *c = line.split()
        paper[(ex, sol, int(n))] = [int(x) for x in c]
    meshes = (9, 27, 81, 243)
    degrees = (2, 3, 4, 5, 6)
    settings = [(nu, om, 1, s0, cg) for nu in (2, 3, 4, 6) for om in (0.8, 0.9, 1.0) for s0 in (1.0, 2.0)
                for cg in (1, 2)]
    out = []
    T0 = time.perf_counter()
    for nu, om, bv, s0, cg in settings:
        counts = {}
        for sol, kind in (("sin_product", 1), ("two_peak", 2)):
            for n in meshes:
                for p in degrees:
                    try:
                        g = hp.Solver(2, n, p, 1.0, p_coarsening=1, h_factor=3, coarsest_n=3, precision=hp.PREC_F64,
                                      nu_pre=nu, nu_post=0, nu_pre_cg=cg, nu_post_cg=cg, omega_dg=om,
                                      block_variant=bv, sigma0=s0)
                    except hp.HpmgError:  # penalty too small: a cell block is not positive definite
                        for ex in ("unprec", "prec"):
                            counts.setdefault((ex, sol, n), []).append(None)
                        continue
                    b = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
                    g.load_vector(kind, 2.0, b)
                    for ex in ("unprec", "prec"):
                        u = torch.zeros_like(b)
                        info, st = g.mgmult(u, b, rtol=1e-7, maxit=1000, exit=ex, check=False)
                        counts.setdefault((ex, sol, n), []).append(info.iterations if st == 0 else None)
                    g.close()
        logs = [abs(math.log(c / q)) for k, cs in counts.items() for c, q in zip(cs, paper[k]) if c]
        dist = statistics.fmean(logs) if logs else None
        out.append({"nu_pre": nu, "nu_post": 0, "omega_dg": om, "block_variant": bv, "sigma0": s0,
                    "nu_q1": [cg, cg],
                    "mean_abs_log_ratio_to_paper": dist, "diverged": sum(1 for cs in counts.values()
                                                                          for c in cs if c is None),
                    "cycles": {f"{e}/{s}/{n}": cs for (e, s, n), cs in counts.items()}})
        _progress(f"nu={nu} omega={om} block={bv} sigma0={s0} q1=({cg},{cg}): distance {dist}")
    best = min((o for o in out if o["mean_abs_log_ratio_to_paper"] is not None and not o["diverged"]),
               key=lambda o: o["mean_abs_log_ratio_to_paper"])
    line = {
        "metric": "paper-mode hp-multigrid cycles to 1e-7 (2D)", "value": None, "unit": "cycles",
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": "2D Poisson, SIPG Q_p on n^2 cells (Gauss-Lobatto nodes), manufactured "
                               "sin(2 pi x)sin(2 pi y) and two-peak solutions, MGMult with nu pre- and zero "
                               "post-smoothing block-Jacobi steps with the interior-cell block (Q1 levels: nu_q1 pre "
                               "and post point-Jacobi steps, omega_CG 2/3), penalty sigma0 (p+1)^2/h, one-step "
                               "DG_p -> Q1, factor-3 h-coarsening to 3^2, FP64",
                   "meshes": list(meshes), "degrees": list(degrees)},
        "settings": out, "closest_to_paper": {k: best[k] for k in ("nu_pre", "omega_dg", "block_variant", "sigma0",
                                                                   "nu_q1", "mean_abs_log_ratio_to_paper")},
        "paper": {f"{e}/{s}/{n}": c for (e, s, n), c in paper.items()},
        "total_s": time.perf_counter() - T0,
    }
    print(json.dumps(line), flush=True)


# --------------------------------------------------------- single problem
def run_single(args):
    import math

    import torch

    import paper_2510_00998_amd as hp
    import synth
    from paper_2510_00998_amd import traffic

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
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    gmx = hp.Solver(dim, n, p, kappa, precision=hp.PREC_F32)
    if args.profile_solve:
        bp = torch.empty(g64.ndof, dtype=torch.float64, device=dev)
        g64.load_vector(fkind, 1.0, bp)
        up = torch.zeros_like(bp)
        out = []
        for _ in range(3):
            up.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info, st = gmx.solve(up, bp, rtol=1e-10, maxit=200, check=False)
            torch.cuda.synchronize()
            out.append({"seconds": time.perf_counter() - t0, "iterations": info.iterations, "status": st})
        print(json.dumps({"profile_solve": out}), flush=True)
        return
    g16 = hp.Solver(dim, n, p, kappa, precision=hp.PREC_F16)
    gb16 = hp.Solver(dim, n, p, kappa, precision=hp.PREC_BF16)
    nd = g64.ndof
    b64 = torch.empty(nd, dtype=torch.float64, device=dev)
    g64.load_vector(fkind, 1.0, b64)
    # sweep inputs per storage type; 16-bit b scaled to mean square
    # lambda = d pi^2 kappa_min (h/N)^d like the solver's 16-bit cycles, so
    # that the iterates stay in FP16 range
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
    # 16-bit storage sweeps with the volume contractions on the matrix cores
    # (the solve uses BF16 operands: FP16 operands of the contractions can
    # overflow under strong coefficient contrast)
    gmf = hp.Solver(dim, n, p, kappa, precision=hp.PREC_BF16, mfma=1)
    mf_in = {name: (torch.zeros(nd, dtype=sweep_in[name][1].dtype, device=dev), sweep_in[name][1],
                    [torch.cuda.Event(enable_timing=True) for _ in range(2)]) for name in ("f16", "bf16")}
    solves = ("fp64", "mixed_f32", "mixed_f16", "mixed_bf16", "mixed_bf16_mfma")
    solver_of = {"fp64": g64, "mixed_f32": gmx, "mixed_f16": g16, "mixed_bf16": gb16, "mixed_bf16_mfma": gmf}
    rc_in = {}
    t_setup_rc = None
    if vark:
        # the same sweeps and mixed solve with the block inverse rebuilt in
        # every traversal from kappa (no stored per-cell eigendata)
        t0 = time.perf_counter()
        grc = hp.Solver(dim, n, p, kappa, block_recompute=1)
        torch.cuda.synchronize()
        t_setup_rc = time.perf_counter() - t0
        rc_in = {name: (torch.zeros(nd, dtype=dt, device=dev), b64.to(dt),
                        [torch.cuda.Event(enable_timing=True) for _ in range(2)])
                 for name, dt in (("f64", torch.float64), ("f32", torch.float32))}
        solves += ("mixed_f32_block_recompute",)
        solver_of["mixed_f32_block_recompute"] = grc
        # split and postpone: stored records, next traversal's rebuilt on a
        # second stream during each sweep
        gsp = hp.Solver(dim, n, p, kappa, block_recompute=2)
        sp_in = {name: (torch.zeros(nd, dtype=dt, device=dev), b64.to(dt),
                        [torch.cuda.Event(enable_timing=True) for _ in range(2)])
                 for name, dt in (("f64", torch.float64), ("f32", torch.float32))}
    else:
        solves += ("mixed_f32_graph",)
        batch1 = hp.Batch([gmx])
    S = args.sweeps

    def sweeps_timed(which=("sw_", "swmf_", "swrc_", "swsp_")):
        out = {}
        for gs, ins, pre in ((g64, sweep_in, "sw_"), (gmf, mf_in, "swmf_")) + (
                ((grc, rc_in, "swrc_"), (gsp, sp_in, "swsp_")) if vark else ()):
            if pre not in which:
                continue
            for uu, bb, evs in ins.values():
                gs.project(uu)
                evs[0].record(stream)
                gs.sweep(uu, bb, S)
                evs[1].record(stream)
        torch.cuda.synchronize()
        for pre, ins in (("sw_", sweep_in), ("swmf_", mf_in), ("swrc_", rc_in)) + ((("swsp_", sp_in),) if vark else ()):
            if pre not in which:
                continue
            for name, (_, _, evs) in ins.items():
                out[pre + name] = evs[0].elapsed_time(evs[1]) * 1e-3 / S
        return out

    if args.profile_sweeps:
        t = sweeps_timed(("swrc_", "swsp_") if (vark and args.block_recompute) else ("sw_", "swmf_"))
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"profile_sweeps": S, "mean_sweep_s": t}), flush=True)
        return

    def step():
        out = sweeps_timed()
        for name in solves:
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "mixed_f32_graph":
                infos, st = batch1.solve([u], [b64], rtol=1e-10, maxit=300, check=False)
                info = infos[0]
            else:
                info, st = solver_of[name].solve(u, b64, rtol=1e-10, maxit=300, check=False)
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0, info.iterations, st,
                         info.final_residual / max(info.initial_residual, 1e-300))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    T = time.perf_counter() - T0

    tsw = {name: _median([r["sw_" + name] for r in res]) for name in sweep_in}
    isz = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
    bysw = {name: traffic.sweep_bytes(dim, n, p, isz[name], per_cell_kappa=vark) for name in sweep_in}
    t64, t32 = tsw["f64"], tsw["f32"]
    by64, by32 = bysw["f64"], bysw["f32"]
    conv = {k: all(r[k][2] == 0 for r in res) for k in solves}
    tmed = {k: _median([r[k][0] for r in res]) for k in solves}
    tt = {k: (tmed[k] if conv[k] else None) for k in solves}
    its = {k: res[-1][k][1] for k in solves}
    final_rel = {k: res[-1][k][3] for k in solves}
    # a solver that stopped at the FP64 evaluation floor of b - A u (status
    # "not converged" with the residual it reached) gets its time to that
    # residual reported separately
    floor = {k: {"seconds": tmed[k], "rel_residual": final_rel[k]} for k in solves if not conv[k]}
    cyc = {"fp64": 8, "mixed_f32": 4, "mixed_f16": 2, "mixed_bf16": 2, "mixed_f32_graph": 4, "mixed_bf16_mfma": 2}
    tts = {}
    for k, isz_c in cyc.items():
        if k in solves and tt.get(k):
            by = traffic.fcg_iteration_bytes(dim, n, p, isz_c) * its[k]
            tts[k] = {"achieved": by / tt[k] / 1e9, "frac": by / tt[k] / 1e9 / HBM_PEAK_GBS,
                      "bytes_per_iteration": traffic.fcg_iteration_bytes(dim, n, p, isz_c)}

    copy_gbs = measured_copy_bandwidth(torch, dev, stream)
    ach64 = by64 / t64 / 1e9
    srcs = ["dg_kernels_impl.hpp"]
    tsum = {2: "sweep_q4_32cube_hbm_traffic.md", 3: "variable_kappa_q3_64cube_hbm_traffic.md",
            5: "sweep_q5_96cube_hbm_traffic.md"}[args.config]
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
                     "frac": ach64 / HBM_PEAK_GBS,
                     "traffic": counter_traffic(tsum, srcs, "traffic_bytes_per_launch_f64"),
                     "kernel": f"k_sweep<double,3,{p + 1},false,{str(vark).lower()},false,false,false> (fused sweep, FP64)",
                     "algorithmic_bytes_per_launch": by64, "mean_launch_s": t64,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": ach64 / copy_gbs},
        "sweep_dofs_per_s": {name: nd / t for name, t in tsw.items()},
        "sweep_roofline": {name: {"achieved": bysw[name] / tsw[name] / 1e9, "frac": bysw[name] / tsw[name] / 1e9 /
                                  HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bysw[name],
                                  "mean_launch_s": tsw[name],
                                  "traffic": counter_traffic(tsum, srcs, f"traffic_bytes_per_launch_{name}")}
                           for name in sweep_in},
        "sweep_matrix_cores_16bit": {
            name: {"dofs_per_s": nd / tmf, "frac": bysw[name] / tmf / 1e9 / HBM_PEAK_GBS, "mean_launch_s": tmf,
                   "traffic": counter_traffic(tsum, srcs, f"traffic_bytes_per_launch_{name}_mfma")}
            for name, tmf in ((nm, _median([r["swmf_" + nm] for r in res])) for nm in mf_in)},
        "time_to_1e-10_s": tt,
        "time_to_attained_residual_s": floor or None,
        "time_to_solution_roofline": tts,
        "solver_iterations": its,
        "converged_by_solver": conv,
        "final_rel_residual_by_solver": final_rel,
        "setup_s": t_setup,
    }
    if vark:
        trc = {name: _median([r["swrc_" + name] for r in res]) for name in rc_in}
        rsum = {3: "variable_kappa_q3_64cube_recompute_hbm_traffic.md", 5: "sweep_q5_96cube_recompute_hbm_traffic.md"}[
            args.config]
        byrc = {name: traffic.sweep_bytes(dim, n, p, isz[name], per_cell_kappa=True, block_recompute=True)
                for name in rc_in}
        line["block_recompute"] = {
            "setup_s": t_setup_rc,
            "sweep_dofs_per_s": {name: nd / t for name, t in trc.items()},
            "sweep_mean_launch_s": trc,
            "sweep_roofline_frac": {name: byrc[name] / trc[name] / 1e9 / HBM_PEAK_GBS for name in rc_in},
            "algorithmic_bytes_per_launch": byrc,
            "traffic": {name: counter_traffic(rsum, srcs, f"traffic_bytes_per_launch_{name}_recompute")
                        for name in rc_in}}
        tsp = {name: _median([r["swsp_" + name] for r in res]) for name in sp_in}
        line["split_and_postpone"] = {
            "sweep_dofs_per_s": {name: nd / t for name, t in tsp.items()},
            "sweep_mean_s": tsp,
            "sweep_roofline_frac_stored_bytes": {name: bysw[name] / tsp[name] / 1e9 / HBM_PEAK_GBS for name in sp_in},
            "traffic_sweep_and_rebuild": {name: counter_traffic(rsum, srcs, f"traffic_bytes_per_launch_{name}_split")
                                          for name in sp_in},
            "note": "mean time per sweep while the next traversal's records are rebuilt on a second stream"}
    print(json.dumps(line), flush=True)


ADAPTIVE_BALLS = ([(0.3, 0.4, 0.5), (0.75, 0.6, 0.5)], [0.25, 0.15])


def adaptive_leaves(n, r=2, max_level=2):
    """Leaves of the adaptive workload: base n^3, cells meeting two balls
    refined by r up to max_level, facet-balanced (synth)."""
    import synth
    return synth.spacetree_leaves(3, n, r, synth.ball_refinement(*ADAPTIVE_BALLS), max_level)


def _adaptive_oracle_baseline(seconds):
    """The oracle on a bounded sample of the adaptive workload: the same
    refinement pattern on 3^3 base cells, assembled SIPG block-Jacobi sweeps
    (dense Cholesky blocks) for about `seconds` on one core, one BLAS thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.adaptive import AdaptiveHierarchy

    leaves = adaptive_leaves(3)
    with threadpool_limits(limits=1):
        H = AdaptiveHierarchy(3, 3, 2, leaves, 4)
        nd = H.fine.ndof
        b = synth.random_rhs(nd, seed=6)
        u = np.zeros_like(b)
        sweeps, t = 0, 0.0
        t0 = time.perf_counter()
        while t < seconds or sweeps < 2:
            u = H.smooth(0, u, b, 1)
            sweeps += 1
            t = time.perf_counter() - t0
    return {"value": nd * sweeps / t, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"same refinement on 3^3 base cells ({len(leaves)} leaves, {nd} DoFs), {sweeps} assembled "
                      f"block-Jacobi sweeps in {t:.1f} s"}


def run_adaptive(args):
    import torch

    import paper_2510_00998_amd as hp
    from paper_2510_00998_amd import traffic

    n, r, p, dim = 16, 2, 4, 3
    cpu = None if args.no_cpu_baseline else _adaptive_oracle_baseline(args.cpu_seconds)
    leaves = adaptive_leaves(n, r)
    counts = traffic.adaptive_facet_counts(dim, n, r, leaves)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t_setup = time.perf_counter()
    g64 = hp.Solver(dim, n, p, 1.0, leaves=leaves, refine=r, precision=hp.PREC_F64)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    gmx = hp.Solver(dim, n, p, 1.0, leaves=leaves, refine=r, precision=hp.PREC_F32)
    nd = g64.ndof
    b64 = torch.empty(nd, dtype=torch.float64, device=dev)
    g64.load_vector(1, 1.0, b64)
    sweep_in = {name: (torch.zeros(nd, dtype=dt, device=dev), b64.to(dt),
                       [torch.cuda.Event(enable_timing=True) for _ in range(2)])
                for name, dt in (("f64", torch.float64), ("f32", torch.float32))}
    u = torch.zeros(nd, dtype=torch.float64, device=dev)
    S = args.sweeps
    solves = {"fp64": g64, "mixed_f32": gmx}

    def sweeps_timed():
        for uu, bb, evs in sweep_in.values():
            g64.project(uu)
            evs[0].record(stream)
            g64.sweep(uu, bb, S)
            evs[1].record(stream)
        torch.cuda.synchronize()
        return {name: evs[0].elapsed_time(evs[1]) * 1e-3 / S for name, (_, _, evs) in sweep_in.items()}

    if args.profile_sweeps:
        t = sweeps_timed()
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"profile_sweeps": S, "mean_sweep_s": t}), flush=True)
        return

    def step():
        out = sweeps_timed()
        for name, g in solves.items():
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info, st = g.solve(u, b64, rtol=1e-10, maxit=300, check=False)
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0, info.iterations, st,
                         info.final_residual / max(info.initial_residual, 1e-300))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    tsw = {name: _median([rr[name] for rr in res]) for name in sweep_in}
    isz = {"f64": 8, "f32": 4}
    bysw = {name: traffic.adaptive_sweep_bytes(dim, n, r, leaves, p, isz[name], counts) for name in sweep_in}
    conv = {k: all(rr[k][2] == 0 for rr in res) for k in solves}
    tt = {k: (_median([rr[k][0] for rr in res]) if conv[k] else None) for k in solves}
    srcs = ["dg_kernels_impl.hpp", "adapt_kernels.hip"]
    tsum = "adaptive_q4_16cube_hbm_traffic.md"
    ach = {name: bysw[name] / tsw[name] / 1e9 for name in sweep_in}
    levels = {int(l): int(c) for l, c in zip(*__import__("numpy").unique(leaves[:, 0], return_counts=True))}
    line = {
        "metric": METRIC,
        "value": nd / tsw["f64"],
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
        "config": {"workload": f"3D SIPG Q{p} on an adaptive spacetree: {n}^3 base cells, cells meeting balls "
                               f"{ADAPTIVE_BALLS[0]} radii {ADAPTIVE_BALLS[1]} refined by {r} up to level 2, "
                               f"facet-balanced: {len(leaves)} leaves {levels}, {nd} DoFs, "
                               f"{counts['interfaces']} hanging facets; u=prod sin(pi x_i); fused sweep + "
                               "hanging-facet remap, hp V(2,2) (p halved, then Q1 on the base mesh), FCG to 1e-10",
                   "dim": dim, "n_base": n, "refine": r, "p": p, "nleaf": len(leaves), "ndof": nd,
                   "hanging_facets": counts["interfaces"], "sweeps_per_step": S},
        "roofline": {"bound": "hbm", "achieved": ach["f64"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach["f64"] / HBM_PEAK_GBS,
                     "traffic": counter_traffic(tsum, srcs, "traffic_bytes_per_launch_f64"),
                     "kernel": f"k_sweep<double,3,{p + 1},false,false,false,false,true> + k_remap<double> "
                               "(fused sweep and hanging-facet remap, FP64)",
                     "algorithmic_bytes_per_launch": bysw["f64"], "mean_launch_s": tsw["f64"]},
        "sweep_dofs_per_s": {name: nd / t for name, t in tsw.items()},
        "sweep_roofline": {name: {"achieved": ach[name], "frac": ach[name] / HBM_PEAK_GBS,
                                  "algorithmic_bytes_per_launch": bysw[name], "mean_launch_s": tsw[name],
                                  "traffic": counter_traffic(tsum, srcs, f"traffic_bytes_per_launch_{name}")}
                           for name in sweep_in},
        "time_to_1e-10_s": tt,
        "solver_iterations": {k: res[-1][k][1] for k in solves},
        "converged_by_solver": conv,
        "final_rel_residual_by_solver": {k: res[-1][k][3] for k in solves},
        "setup_s": t_setup,
        "cpu_baseline": cpu,
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
    elif args.config == 4:
        run_batched(args)
    elif args.config == 6:
        run_adaptive(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
