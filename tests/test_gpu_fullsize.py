"""Parity at the full workload sizes, in the launch configuration bench.py
times, on sampled cells the oracle evaluates one block row at a time
(apply_A and one block-Jacobi sweep), plus size-independent properties of
the mixed-precision solve."""
import numpy as np
import pytest

import synth
from oracle import SIPG
from tests.gpu_common import log, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WORKLOADS = {
    # name: dim, n, p, kappa factory
    "q4_32cube_const": (3, 32, 4, lambda: 1.0),
    "q3_64cube_loguniform": (3, 64, 3, lambda: synth.kappa_log_uniform(3, 64, seed=1003)),
    "q5_96cube_lognormal": (3, 96, 5, lambda: synth.kappa_log_normal(3, 96, seed=1005)),
}


def _sample_cells(n, dim, count, seed):
    """Corners, edge and face cells plus random interior cells."""
    ncell = n ** dim
    corners = [0, n - 1, n * (n - 1), n * n - 1, ncell - 1, ncell - n, ncell - n * n, ncell - n * n + n - 1]
    rnd = (synth.uniform(seed, count) * ncell).astype(np.int64)
    mids = [n // 2, n * (n // 2), n * n * (n // 2) + n * (n // 2) + n // 2]
    return np.unique(np.concatenate([corners, mids, rnd]))


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_apply_and_sweep_sampled(name):
    import paper_2510_00998_amd as hp
    dim, n, p, kf = WORKLOADS[name]
    kappa = kf()
    log(f"full-size {name}: dim={dim} n={n} p={p}")
    s = SIPG(dim, n, p, kappa)  # reference blocks only; no global assembly
    g = hp.Solver(dim, n, p, kappa)
    nd = g.ndof
    cells = _sample_cells(n, dim, 96, seed=7)
    u0 = synth.random_vector(nd, seed=11)
    b = synth.random_rhs(nd, seed=12)
    y_ref = s.apply_rows(cells, u0)
    # one block-Jacobi step on the sampled cells
    blocks = s._diag_blocks_for(cells)
    r = b.reshape(s.ncell, s.nd)[cells] - y_ref
    u1_ref = u0.reshape(s.ncell, s.nd)[cells] + 0.7 * np.linalg.solve(blocks, r[..., None])[..., 0]
    for dt, tol_a, tol_s in ((torch.float64, 1e-12, 1e-11), (torch.float32, 1e-5, 1e-5)):
        ud = torch.tensor(u0, dtype=dt, device="cuda")
        yd = torch.empty_like(ud)
        g.apply_A(ud, yd)
        y = to_host(yd).reshape(s.ncell, s.nd)[cells]
        ref = y_ref if dt == torch.float64 else s.apply_rows(cells, u0.astype(np.float32).astype(np.float64))
        ea = np.abs(y - ref).max() / np.abs(ref).max()
        bd = torch.tensor(b, dtype=dt, device="cuda")
        g.smooth(ud, bd, 1)
        u1 = to_host(ud).reshape(s.ncell, s.nd)[cells]
        es = np.abs(u1 - u1_ref).max() / np.abs(u1_ref).max()
        log(f"  {dt}: apply rel err {ea:.2e}, sweep rel err {es:.2e} on {len(cells)} cells")
        assert ea <= tol_a
        assert es <= tol_s
        del ud, yd, bd
    g.close()


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("name", ["q4_32cube_const", "q3_64cube_loguniform"])
def test_fullsize_mixed_solve_residual(name, prec):
    # the true FP64 residual of the mixed-precision solution (FP32 cycle, or
    # FP32 cycle with 16-bit storage of the finest level) meets the 1e-10
    # relative tolerance (checked with the parity-tested FP64 apply)
    import paper_2510_00998_amd as hp
    dim, n, p, kf = WORKLOADS[name]
    kappa = kf()
    pr = {"f32": hp.PREC_F32, "f16": hp.PREC_F16, "bf16": hp.PREC_BF16}[prec]
    log(f"{name} {prec}")
    g = hp.Solver(dim, n, p, kappa, precision=pr)
    b = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    g.load_vector(0, 1.0, b)
    u = torch.zeros_like(b)
    info, st = g.solve(u, b, rtol=1e-10, maxit=200)
    y = torch.empty_like(u)
    g.apply_A(u, y)
    rel = float(torch.linalg.vector_norm(b - y) / torch.linalg.vector_norm(b))
    log(f"  {name} {prec}: {info.iterations} its, true rel residual {rel:.2e}")
    assert st == 0 and rel <= 2e-10
    g.close()


def test_fullsize_batched_workload():
    # the 64 problems x 4 RHS batched workload at full size (as the bench runs
    # it): every segment's true FP64 residual (parity-tested apply) meets the
    # tolerance, and the oracle's own residual on the smallest problems
    import paper_2510_00998_amd as hp
    probs = synth.batched_problem_list()
    R = 4
    solvers = [hp.Solver(3, n, p, 1.0, max_rhs=R) for n, p in probs]
    batch = hp.Batch(solvers)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1004)
    bs = [torch.randn(R * s.ndof, dtype=torch.float64, device="cuda", generator=gen) for s in solvers]
    us = [torch.zeros_like(b) for b in bs]
    infos, st = batch.solve(us, bs, rtol=1e-10, maxit=200, nrhs=R)
    log(f"batched 64x4: status {st}, max iterations {max(i.iterations for i in infos)}")
    assert st == 0
    worst = 0.0
    for s, u, b in zip(solvers, us, bs):
        y = torch.empty_like(u)
        s.apply_A(u, y, nrhs=R)
        for r in range(R):
            sl = slice(r * s.ndof, (r + 1) * s.ndof)
            worst = max(worst, float(torch.linalg.vector_norm(b[sl] - y[sl]) / torch.linalg.vector_norm(b[sl])))
    log(f"  worst true relative residual {worst:.2e}")
    assert worst <= 2e-10
    small = sorted(range(len(probs)), key=lambda j: solvers[j].ndof)[:2]
    for j in small:
        n, p = probs[j]
        A = SIPG(3, n, p).A
        u, b = to_host(us[j]), to_host(bs[j])
        nd = solvers[j].ndof
        rr = max(np.linalg.norm(b[r * nd:(r + 1) * nd] - A @ u[r * nd:(r + 1) * nd]) /
                 np.linalg.norm(b[r * nd:(r + 1) * nd]) for r in range(R))
        log(f"  problem {j} (n={n}, p={p}): oracle residual {rr:.2e}")
        assert rr <= 2e-10


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_variant_sweeps_sampled(name):
    # one sweep with 16-bit storage of u and traces (FP32 arithmetic) on all
    # three workloads, and, for the variable-coefficient ones, one sweep with
    # the block data rebuilt in the traversal (block_recompute = 1) and with
    # split-and-postpone rebuilds (block_recompute = 2), against the oracle's
    # block-Jacobi step on sampled cells
    import paper_2510_00998_amd as hp
    dim, n, p, kf = WORKLOADS[name]
    kappa = kf()
    vark = not isinstance(kappa, float)
    log(f"full-size variants {name}: dim={dim} n={n} p={p}")
    s = SIPG(dim, n, p, kappa)
    cells = _sample_cells(n, dim, 64, seed=9)
    u0 = synth.random_vector(s.ndof, seed=21)
    b = synth.random_rhs(s.ndof, seed=22)
    blocks = s._diag_blocks_for(cells)

    def step_ref(uu, bb):
        r = bb.reshape(s.ncell, s.nd)[cells] - s.apply_rows(cells, uu)
        return uu.reshape(s.ncell, s.nd)[cells] + 0.7 * np.linalg.solve(blocks, r[..., None])[..., 0]

    g = hp.Solver(dim, n, p, kappa)
    # 16-bit storage: inputs rounded to the format; one sweep stores u and
    # the traces once (about 2 unit roundoffs of the format, bound 4)
    for dt, u in ((torch.float16, 2.0 ** -11), (torch.bfloat16, 2.0 ** -8)):
        ud = torch.tensor(u0, dtype=torch.float64, device="cuda").to(dt)
        bd = torch.tensor(b, dtype=torch.float64, device="cuda").to(dt)
        ur, br = to_host(ud), to_host(bd)
        ref = step_ref(ur, br)
        g.smooth(ud, bd, 1)
        got = to_host(ud).reshape(s.ncell, s.nd)[cells]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        log(f"  {dt}: sweep rel err {err:.2e} on {len(cells)} cells")
        assert err <= 4 * u
        del ud, bd
    g.close()
    if vark:
        ref = step_ref(u0, b)
        for mode in (1, 2):
            gr = hp.Solver(dim, n, p, kappa, block_recompute=mode)
            for dt, tol in ((torch.float64, 1e-11), (torch.float32, 1e-5)):
                ud = torch.tensor(u0, dtype=dt, device="cuda")
                bd = torch.tensor(b, dtype=dt, device="cuda")
                gr.smooth(ud, bd, 1)
                got = to_host(ud).reshape(s.ncell, s.nd)[cells]
                err = np.abs(got - ref).max() / np.abs(ref).max()
                log(f"  block_recompute={mode} {dt}: sweep rel err {err:.2e}")
                assert err <= tol
                del ud, bd
            gr.close()


def test_q4_manufactured_solution_rate():
    # the Q4 workload's path (FP32 cycle inside FP64 FCG to 1e-10) on 8^3,
    # 16^3, 32^3: the L2 error of u = prod sin(pi x_i) decreases at the rate
    # p + 1 = 5, and at 32^3 it equals the error of a far tighter FP64-cycle
    # solve within 1% (the solve error is below the discretisation error)
    import paper_2510_00998_amd as hp
    from oracle import manufactured as mf
    uex, _ = mf.sin_product(3, 1)
    errs = {}
    for n in (8, 16, 32):
        s = SIPG(3, n, 4)
        g = hp.Solver(3, n, 4, 1.0)
        bd = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        g.load_vector(1, 1.0, bd)
        x = torch.zeros_like(bd)
        info, st = g.solve(x, bd, rtol=1e-10, maxit=100)
        assert st == 0
        errs[n] = s.l2_error(to_host(x), uex)
        log(f"Q4 n={n}: L2 error {errs[n]:.4e} ({info.iterations} its)")
        if n == 32:
            g64 = hp.Solver(3, n, 4, 1.0, precision=hp.PREC_F64)
            x2 = torch.zeros_like(bd)
            g64.solve(x2, bd, rtol=1e-13, maxit=200, check=False)
            e_tight = s.l2_error(to_host(x2), uex)
            log(f"  32^3 tight FP64 solve: L2 error {e_tight:.4e}")
            assert abs(errs[n] - e_tight) <= 0.01 * e_tight
        g.close()
    for a, b_ in ((8, 16), (16, 32)):
        rate = np.log2(errs[a] / errs[b_])
        log(f"  rate {a}->{b_}: {rate:.3f}")
        assert abs(rate - 5.0) <= 0.25
