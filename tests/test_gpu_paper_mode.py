"""Paper-mode options through the C ABI against the oracle: one-step
p-coarsening DG_p -> Q1, factor-3 h-coarsening of the Q1 levels, the
stationary MGMult iteration with the unpreconditioned and the
preconditioned exit (Sections 5.1.1, 5.2), and the two-peak load vector."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy, HierarchyOptions, manufactured as mf
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # dim, n, p, kappa kind, p_coarsening (0 halve, 1 direct), h_factor
    (2, 9, 4, "const", 1, 3),
    (2, 10, 5, "var", 1, 3),
    (2, 27, 2, "const", 1, 3),
    (2, 12, 4, "var", 0, 3),
    (3, 6, 4, "const", 1, 3),
    (3, 4, 3, "var", 1, 2),
    (3, 5, 6, "const", 1, 2),
]


def _kappa(dim, n, kind, seed=300):
    return 1.3 if kind == "const" else synth.kappa_log_uniform(dim, n, seed=seed)


def _opts(pc, hf):
    return HierarchyOptions(p_coarsening="direct" if pc else "halve", h_factor=hf)


@pytest.mark.parametrize("dim,n,p,kind,pc,hf", CASES)
def test_vcycle_paper_options(dim, n, p, kind, pc, hf):
    import paper_2510_00998_amd as hp
    log(f"vcycle dim={dim} n={n} p={p} kappa={kind} direct={pc} factor={hf}")
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind), opts=_opts(pc, hf))
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=41)
    b = synth.random_rhs(nd, seed=42)
    ref = H.vcycle(0, u0.copy(), b)
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind), p_coarsening=pc, h_factor=hf)
    for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):  # FP32: about 10 u32 per traversal
        ud, bd = to_dev(u0, dt), to_dev(b, dt)
        g.vcycle(ud, bd)
        err = rel_err(to_host(ud), ref)
        log(f"  {dt}: rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("exit", ["unprec", "prec"])
@pytest.mark.parametrize("dim,n,p,sol", [(2, 9, 3, "sin"), (2, 27, 2, "two_peak"), (2, 9, 5, "two_peak")])
def test_mgmult_matches_oracle(dim, n, p, sol, exit):
    import paper_2510_00998_amd as hp
    log(f"mgmult {exit} dim={dim} n={n} p={p} {sol}")
    opts = HierarchyOptions(p_coarsening="direct", h_factor=3, coarsest_n=3)
    H = Hierarchy(dim, n, p, opts=opts)
    f = mf.sin_product(2, 2)[1] if sol == "sin" else mf.two_peak()[1]
    b = H.fine.load_vector(f)
    _, hist, phist = H.mgmult(b, rtol=1e-7, maxit=300, exit=exit)
    ref = (np.array(hist[1:]) / hist[0]) if exit == "unprec" else np.array(phist) / phist[0]
    g = hp.Solver(dim, n, p, 1.0, p_coarsening=1, h_factor=3, coarsest_n=3, precision=hp.PREC_F64)
    bd = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    g.load_vector(1 if sol == "sin" else 2, 2.0, bd)
    assert rel_err(to_host(bd), b) <= 1e-13
    ud = torch.zeros_like(bd)
    info, st = g.mgmult(ud, bd, rtol=1e-7, maxit=300, exit=exit)
    got = np.array(info.residual_history[:info.iterations])
    log(f"  cycles gpu {info.iterations} oracle {len(ref)}")
    assert st == 0
    assert info.iterations == len(ref)
    assert np.abs(got - ref).max() <= 1e-7 * np.abs(ref).max()


def test_mgmult_reduced_precision_cycles_converge():
    import paper_2510_00998_amd as hp
    s = SIPG(2, 27, 3)
    b = s.load_vector(mf.two_peak()[1])
    for pr in (hp.PREC_F32, hp.PREC_F16, hp.PREC_BF16):
        g = hp.Solver(2, 27, 3, 1.0, p_coarsening=1, h_factor=3, coarsest_n=3, precision=pr)
        bd = to_dev(b, torch.float64)
        ud = torch.zeros_like(bd)
        info, st = g.mgmult(ud, bd, rtol=1e-7, maxit=300)
        rr = np.linalg.norm(b - s.A @ to_host(ud)) / np.linalg.norm(b)
        log(f"  precision {pr}: {info.iterations} cycles, oracle residual {rr:.2e}")
        assert st == 0 and rr <= 1.5e-7
