"""16-bit storage (FP16 / BF16) of the finest level, FP32 arithmetic: the
sweep and the V-cycle against the oracle on the rounded inputs, and the
mixed solves (FP64 outer iteration) to the full tolerance, through the C ABI."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # dim, n, p, kappa kind
    (2, 16, 2, "const"),
    (2, 5, 4, "var"),
    (3, 5, 2, "const"),
    (3, 4, 3, "var"),
    (3, 4, 4, "const"),
    (3, 3, 5, "var"),
    (3, 3, 1, "var"),
    (3, 2, 8, "const"),
]

# Relative max-norm tolerances.  Every sweep stores u and its traces once in
# 16 bits (unit roundoff u16 = 2^-11 for FP16, 2^-8 for BF16) and the
# FP32 arithmetic adds far less; three sweeps reach the result through three
# roundings of u (3 u16), a V-cycle through four (two pre-smoothing sweeps,
# the prolongation and the post-smoothing; the coarse levels run in FP32).
TOL = {"f16": {"smooth": 3 * 2.0 ** -11, "vcycle": 4 * 2.0 ** -11},
       "bf16": {"smooth": 3 * 2.0 ** -8, "vcycle": 4 * 2.0 ** -8}}


def _kappa(dim, n, kind, seed=100):
    if kind == "const":
        return 2.5
    return synth.kappa_log_uniform(dim, n, seed=seed)


def _dt(name):
    return torch.float16 if name == "f16" else torch.bfloat16


def _rounded(x, name):
    """x rounded to the 16-bit format (host), as float64."""
    return torch.tensor(x, dtype=torch.float64).to(_dt(name)).double().numpy()


@pytest.mark.parametrize("name", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_smooth_16bit_storage(dim, n, p, kind, name):
    import paper_2510_00998_amd as hp
    log(f"smooth {name} dim={dim} n={n} p={p} kappa={kind}")
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = _rounded(synth.random_vector(nd, seed=7), name)
    b = _rounded(synth.random_rhs(nd, seed=8), name)
    ref = H.smooth(0, u0.copy(), b, 3)
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind))
    ud, bd = to_dev(u0, _dt(name)), to_dev(b, _dt(name))
    g.smooth(ud, bd, 3)
    err = rel_err(to_host(ud), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[name]["smooth"]


@pytest.mark.parametrize("name", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_vcycle_16bit_storage(dim, n, p, kind, name):
    import paper_2510_00998_amd as hp
    log(f"vcycle {name} dim={dim} n={n} p={p} kappa={kind}")
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = _rounded(synth.random_vector(nd, seed=17), name)
    b = _rounded(synth.random_rhs(nd, seed=18), name)
    ref = H.vcycle(0, u0.copy(), b)
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind))
    ud, bd = to_dev(u0, _dt(name)), to_dev(b, _dt(name))
    g.vcycle(ud, bd)
    err = rel_err(to_host(ud), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[name]["vcycle"]


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", [(2, 16, 2, "const"), (3, 4, 3, "var"), (3, 5, 4, "const")])
def test_solve_16bit_cycle_reaches_tolerance(dim, n, p, kind, prec):
    import paper_2510_00998_amd as hp
    log(f"solve {prec} dim={dim} n={n} p={p} kappa={kind}")
    s = SIPG(dim, n, p, _kappa(dim, n, kind))
    b = synth.random_rhs(s.ndof, seed=33)
    pr = hp.PREC_F16 if prec == "f16" else hp.PREC_BF16
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind), precision=pr)
    ud, bd = torch.zeros(s.ndof, dtype=torch.float64, device="cuda"), to_dev(b, torch.float64)
    info, st = g.solve(ud, bd, rtol=1e-10, maxit=200)
    u = to_host(ud)
    rr = np.linalg.norm(b - s.A @ u) / np.linalg.norm(b)
    log(f"  its {info.iterations} oracle residual {rr:.3e}")
    assert st == 0
    assert rr <= 2e-10


def test_apply_rejects_16bit():
    import paper_2510_00998_amd as hp
    g = hp.Solver(3, 3, 2, 1.0)
    u = torch.zeros(g.ndof, dtype=torch.float16, device="cuda")
    with pytest.raises(hp.HpmgError):
        g.apply_A(u, u.clone())
