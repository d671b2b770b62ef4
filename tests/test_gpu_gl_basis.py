"""Gauss-Legendre nodes (options.basis = 1: diagonal mass, dense facet value
functionals) through the C ABI against the oracle assembled in the same
basis: apply, block-Jacobi sweeps, V-cycle, solve, load vector."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy, HierarchyOptions, manufactured as mf
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    (2, 5, 3, "const"),
    (2, 4, 4, "var"),
    (2, 3, 7, "const"),
    (3, 3, 2, "var"),
    (3, 4, 4, "const"),
    (3, 3, 5, "var"),
    (3, 3, 1, "const"),
    (3, 2, 8, "var"),
]


def _kappa(dim, n, kind, seed=500):
    return 0.8 if kind == "const" else synth.kappa_log_uniform(dim, n, seed=seed)


@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_gl_apply_smooth_vcycle(dim, n, p, kind):
    import paper_2510_00998_amd as hp
    log(f"GL dim={dim} n={n} p={p} kappa={kind}")
    k = _kappa(dim, n, kind)
    H = Hierarchy(dim, n, p, k, opts=HierarchyOptions(basis="gl"))
    A = H.levels[0].A
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=51)
    b = synth.random_rhs(nd, seed=52)
    g = hp.Solver(dim, n, p, k, basis=1)
    for dt, ta, ts, tv in ((torch.float64, 1e-12, 1e-11, 1e-10), (torch.float32, 1e-5, 1e-5, 1e-5)):
        ud = to_dev(u0, dt)
        yd = torch.empty_like(ud)
        g.apply_A(ud, yd)
        ref = A @ (u0 if dt == torch.float64 else u0.astype(np.float32).astype(np.float64))
        ea = rel_err(to_host(yd), ref)
        ud, bd = to_dev(u0, dt), to_dev(b, dt)
        g.smooth(ud, bd, 3)
        es = rel_err(to_host(ud), H.smooth(0, u0.copy(), b, 3))
        ud = to_dev(u0, dt)
        g.vcycle(ud, bd)
        ev = rel_err(to_host(ud), H.vcycle(0, u0.copy(), b))
        log(f"  {dt}: apply {ea:.2e} smooth {es:.2e} vcycle {ev:.2e}")
        assert ea <= ta and es <= ts and ev <= tv


@pytest.mark.parametrize("dim,n,p", [(2, 6, 3), (3, 3, 4)])
def test_gl_solve_and_load_vector(dim, n, p):
    import paper_2510_00998_amd as hp
    s = SIPG(dim, n, p, basis="gl")
    _, f = mf.sin_product(dim, 1)
    ref = s.load_vector(f)
    g = hp.Solver(dim, n, p, 1.0, basis=1)
    bd = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    g.load_vector(1, 1.0, bd)
    assert rel_err(to_host(bd), ref) <= 1e-13
    for pr in (hp.PREC_F64, hp.PREC_F32):
        g = hp.Solver(dim, n, p, 1.0, basis=1, precision=pr)
        ud = torch.zeros_like(bd)
        info, st = g.solve(ud, bd, rtol=1e-10, maxit=100)
        rr = np.linalg.norm(ref - s.A @ to_host(ud)) / np.linalg.norm(ref)
        log(f"  GL solve precision {pr}: {info.iterations} its, oracle residual {rr:.2e}")
        assert st == 0 and rr <= 2e-10
