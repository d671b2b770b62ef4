"""GPU parity of the HIP path (through the C ABI) against the CPU oracle on
the same seeded inputs, element by element, on meshes that span several
blocks and a ragged last block."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy, HierarchyOptions, manufactured as mf
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# FP32 against the FP64 oracle: inputs rounded to FP32 (u32 = 2^-24) and
# about 10 u32 of arithmetic error per fine-level traversal (the
# sum-factorised contractions sum N terms per stage over 2d stages); three
# sweeps or one V-cycle (about eight fine-level traversals) stay below 1e-5.
TOL32_SMOOTH = 1e-5
TOL32_VCYCLE = 1e-5

CASES = [
    # dim, n, p, kappa kind
    (2, 5, 1, "const"),
    (2, 16, 2, "const"),
    (2, 7, 3, "var"),
    (2, 3, 8, "var"),
    (3, 3, 1, "var"),
    (3, 6, 1, "const"),
    (3, 5, 2, "const"),
    (3, 4, 3, "var"),
    (3, 4, 4, "const"),
    (3, 3, 5, "var"),
    (3, 2, 7, "const"),
    (3, 3, 6, "const"),
    (3, 2, 8, "var"),
]


def _kappa(dim, n, kind, seed=100):
    if kind == "const":
        return 2.5
    return synth.kappa_log_uniform(dim, n, seed=seed)


def _solver(dim, n, p, kind, **opt):
    import paper_2510_00998_amd as hp
    return hp.Solver(dim, n, p, _kappa(dim, n, kind), **opt)


@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_apply_A_fp64_fp32(dim, n, p, kind):
    log(f"apply_A dim={dim} n={n} p={p} kappa={kind}")
    s = SIPG(dim, n, p, _kappa(dim, n, kind))
    u = synth.random_vector(s.ndof, seed=1000 + p)
    y_ref = s.A @ u
    g = _solver(dim, n, p, kind)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        ud = to_dev(u, dt)
        yd = torch.empty_like(ud)
        g.apply_A(ud, yd)
        ref = y_ref if dt == torch.float64 else s.A @ u.astype(np.float32).astype(np.float64)
        err = rel_err(to_host(yd), ref)
        log(f"  {dt}: rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_smooth_matches_block_jacobi(dim, n, p, kind):
    log(f"smooth dim={dim} n={n} p={p} kappa={kind}")
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=7)
    b = synth.random_rhs(nd, seed=8)
    ref = H.smooth(0, u0.copy(), b, 3)
    g = _solver(dim, n, p, kind)
    ud, bd = to_dev(u0, torch.float64), to_dev(b, torch.float64)
    g.smooth(ud, bd, 3)
    err = rel_err(to_host(ud), ref)
    log(f"  fp64 rel err {err:.3e}")
    assert err <= 1e-11
    ud, bd = to_dev(u0, torch.float32), to_dev(b, torch.float32)
    g.smooth(ud, bd, 3)
    err = rel_err(to_host(ud), ref)
    log(f"  fp32 rel err {err:.3e}")
    assert err <= TOL32_SMOOTH


@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_vcycle_matches_oracle(dim, n, p, kind):
    log(f"vcycle dim={dim} n={n} p={p} kappa={kind}")
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=17)
    b = synth.random_rhs(nd, seed=18)
    ref = H.vcycle(0, u0.copy(), b)
    g = _solver(dim, n, p, kind)
    ud, bd = to_dev(u0, torch.float64), to_dev(b, torch.float64)
    g.vcycle(ud, bd)
    err = rel_err(to_host(ud), ref)
    log(f"  fp64 rel err {err:.3e}")
    assert err <= 1e-10
    ud, bd = to_dev(u0, torch.float32), to_dev(b, torch.float32)
    g.vcycle(ud, bd)
    err = rel_err(to_host(ud), ref)
    log(f"  fp32 rel err {err:.3e}")
    assert err <= TOL32_VCYCLE


@pytest.mark.parametrize("dim,n,p,kind", [(2, 16, 2, "const"), (3, 4, 3, "var"), (3, 5, 4, "const")])
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_reaches_tolerance(dim, n, p, kind, prec):
    log(f"solve dim={dim} n={n} p={p} kappa={kind} prec={prec}")
    s = SIPG(dim, n, p, _kappa(dim, n, kind))
    b = synth.random_rhs(s.ndof, seed=33)
    g = _solver(dim, n, p, kind, precision=prec)
    ud, bd = torch.zeros(s.ndof, dtype=torch.float64, device="cuda"), to_dev(b, torch.float64)
    info, st = g.solve(ud, bd, rtol=1e-10, maxit=100)
    u = to_host(ud)
    rr = np.linalg.norm(b - s.A @ u) / np.linalg.norm(b)
    log(f"  its {info.iterations} oracle residual {rr:.3e}")
    assert st == 0
    assert rr <= 2e-10


@pytest.mark.parametrize("dim,n,p", [(2, 16, 2), (3, 4, 4), (3, 3, 3)])
def test_load_vector_matches_oracle(dim, n, p):
    s = SIPG(dim, n, p)
    _, f = mf.sin_product(dim, 1)
    ref = s.load_vector(f)
    g = _solver(dim, n, p, "const")
    bd = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    g.load_vector(1, 1.0, bd)
    assert rel_err(to_host(bd), ref) <= 1e-13
    ref1 = s.load_vector(mf.constant(1.0))
    g.load_vector(0, 1.0, bd)
    assert rel_err(to_host(bd), ref1) <= 1e-13
