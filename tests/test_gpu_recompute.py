"""Block inverse rebuilt in every traversal (block_recompute = 1, variable
kappa): the kernels form each cell's fast-diagonalisation data from kappa by
a Jacobi eigensolve instead of reading stored eigendata.  Checked element by
element against the CPU oracle (assembled operator, dense-Cholesky block
Jacobi, V-cycle) and against the stored-eigendata path on the same inputs."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # dim, n, p: several blocks, full blocks and a ragged last block, p up to
    # 8 (N = 9); 3D degree 2 has a partial last wave in a full block
    (2, 7, 3),
    (2, 6, 2),
    (2, 3, 8),
    (3, 3, 1),
    (3, 5, 2),
    (3, 4, 3),
    (3, 5, 4),
    (3, 3, 5),
    (3, 2, 7),
]


def _kappa(dim, n, seed=300):
    return synth.kappa_log_uniform(dim, n, seed=seed)


def _solvers(dim, n, p, **opt):
    import paper_2510_00998_amd as hp
    k = _kappa(dim, n)
    return hp.Solver(dim, n, p, k, block_recompute=1, **opt), hp.Solver(dim, n, p, k, **opt)


@pytest.mark.parametrize("dim,n,p", CASES)
def test_recompute_apply_and_sweeps(dim, n, p):
    log(f"recompute apply/smooth dim={dim} n={n} p={p}")
    H = Hierarchy(dim, n, p, _kappa(dim, n))
    A = H.fine.A
    nd = H.fine.ndof
    u = synth.random_vector(nd, seed=2000 + p)
    b = synth.random_rhs(nd, seed=2100 + p)
    gr, gs = _solvers(dim, n, p)
    for dt, tol_a, tol_s, tol_x in ((torch.float64, 1e-12, 1e-11, 1e-12), (torch.float32, 1e-5, 1e-5, 1e-5)):
        ud = to_dev(u, dt)
        yr, ys = torch.empty_like(ud), torch.empty_like(ud)
        gr.apply_A(ud, yr)
        gs.apply_A(ud, ys)
        ref = A @ (u if dt == torch.float64 else u.astype(np.float32).astype(np.float64))
        e_or, e_rs = rel_err(to_host(yr), ref), rel_err(to_host(yr), to_host(ys))
        log(f"  {dt} apply: vs oracle {e_or:.3e}, vs stored eigendata {e_rs:.3e}")
        assert e_or <= tol_a and e_rs <= tol_x
        ur, us = to_dev(u, dt), to_dev(u, dt)
        bd = to_dev(b, dt)
        gr.smooth(ur, bd, 3)
        gs.smooth(us, bd, 3)
        ref = H.smooth(0, u.copy(), b, 3)
        e_or, e_rs = rel_err(to_host(ur), ref), rel_err(to_host(ur), to_host(us))
        log(f"  {dt} 3 sweeps: vs oracle {e_or:.3e}, vs stored eigendata {e_rs:.3e}")
        assert e_or <= tol_s and e_rs <= 10 * tol_x


@pytest.mark.parametrize("dim,n,p", [(2, 7, 3), (3, 4, 3), (3, 3, 5), (3, 5, 4)])
def test_recompute_vcycle_and_solve(dim, n, p):
    log(f"recompute vcycle/solve dim={dim} n={n} p={p}")
    H = Hierarchy(dim, n, p, _kappa(dim, n))
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=2200)
    b = synth.random_rhs(nd, seed=2300)
    ref = H.vcycle(0, u0.copy(), b)
    gr, _ = _solvers(dim, n, p)
    ud, bd = to_dev(u0, torch.float64), to_dev(b, torch.float64)
    gr.vcycle(ud, bd)
    err = rel_err(to_host(ud), ref)
    log(f"  fp64 vcycle vs oracle {err:.3e}")
    assert err <= 1e-10
    s = SIPG(dim, n, p, _kappa(dim, n))
    for prec in (0, 1):
        g, _ = _solvers(dim, n, p, precision=prec)
        ud = torch.zeros(nd, dtype=torch.float64, device="cuda")
        info, st = g.solve(ud, bd, rtol=1e-10, maxit=200)
        rr = np.linalg.norm(b - s.A @ to_host(ud)) / np.linalg.norm(b)
        log(f"  solve precision {prec}: its {info.iterations}, oracle residual {rr:.3e}")
        assert st == 0 and rr <= 2e-10


def test_recompute_16bit_storage_sweep():
    dim, n, p = 3, 4, 4
    log(f"recompute fp16 sweep dim={dim} n={n} p={p}")
    H = Hierarchy(dim, n, p, _kappa(dim, n))
    nd = H.fine.ndof
    u = synth.random_vector(nd, seed=2400)
    b = synth.random_rhs(nd, seed=2500)
    ref = H.smooth(0, u.copy(), b, 2)
    gr, _ = _solvers(dim, n, p)
    ud, bd = to_dev(u, torch.float16), to_dev(b, torch.float16)
    gr.smooth(ud, bd, 2)
    err = rel_err(to_host(ud), ref)
    log(f"  fp16 storage, 2 sweeps vs oracle {err:.3e}")
    assert err <= 1.5e-3  # about one FP16 rounding (u16 = 2^-11) of u per sweep


@pytest.mark.parametrize("dim,n,p", [(2, 7, 3), (3, 4, 3), (3, 5, 4), (3, 3, 5), (3, 5, 2)])
def test_split_and_postpone_sweeps(dim, n, p):
    """block_recompute = 2: each sweep reads stored records while the next
    traversal's records are rebuilt on a second stream.  FP64: the rebuild
    is the setup's eigensolve, so the sweeps equal the stored-record sweeps
    bit for bit; FP32 (rebuilt in FP32) and FP16 storage match the oracle.
    A sweep count above two exercises the buffer rotation, hpmg_sweep the
    continuation with the handle's current records."""
    import paper_2510_00998_amd as hp
    log(f"split-and-postpone sweeps dim={dim} n={n} p={p}")
    H = Hierarchy(dim, n, p, _kappa(dim, n))
    nd = H.fine.ndof
    u0 = synth.random_vector(nd, seed=2600 + p)
    b = synth.random_rhs(nd, seed=2700 + p)
    ref = H.smooth(0, u0.copy(), b, 5)
    k = _kappa(dim, n)
    gsp = hp.Solver(dim, n, p, k, block_recompute=2)
    gst = hp.Solver(dim, n, p, k)
    ua, ub = to_dev(u0, torch.float64), to_dev(u0, torch.float64)
    bd = to_dev(b, torch.float64)
    gsp.smooth(ua, bd, 3)
    gsp.sweep(ua, bd, 2)
    gst.smooth(ub, bd, 5)
    assert torch.equal(ua, ub)
    err = rel_err(to_host(ua), ref)
    log(f"  fp64 5 sweeps vs oracle {err:.3e}")
    assert err <= 1e-11
    u32, b32 = to_dev(u0, torch.float32), to_dev(b, torch.float32)
    gsp.smooth(u32, b32, 5)
    err = rel_err(to_host(u32), ref)
    log(f"  fp32 5 sweeps vs oracle {err:.3e}")
    assert err <= 1e-5
    # the operator is unchanged: apply and a V-cycle after split sweeps
    y = torch.empty_like(ua)
    gsp.apply_A(ua, y)
    assert rel_err(to_host(y), H.fine.A @ to_host(ua)) <= 1e-12
