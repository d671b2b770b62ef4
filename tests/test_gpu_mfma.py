"""16-bit storage sweeps with the volume contractions on the matrix cores
(hpmg_options.mfma = 1: v_mfma_f32_16x16x16 with FP16 or BF16 operands, FP32
accumulation) through the C ABI, against the FP64 oracle on the same seeded
inputs (rounded to the storage format), and against the vector-unit sweep of
the same storage format."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy
from tests.gpu_common import log, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# Relative max-norm tolerances in units of the format's unit roundoff u
# (2^-11 FP16, 2^-8 BF16).  A sweep rounds the operands of each of its six
# contraction stages (data and matrix entries, about 2 u per stage) besides
# storing u once: about 13 u per sweep, 39 u for three sweeps; a V-cycle has
# four finest-level sweeps (the coarse levels run in FP32).
U = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
K_SMOOTH, K_VCYCLE = 40, 60

CASES = [(3, 4, 1, "const"), (3, 5, 2, "var"), (3, 4, 3, "const"), (3, 4, 4, "var"), (3, 3, 4, "const"),
         (3, 3, 5, "var"), (3, 2, 6, "const"), (3, 2, 7, "var"), (3, 2, 8, "var")]

# FP16 inputs are scaled by 2^-6 (exactly): with kappa up to 100 and degree 7
# or 8 the facet fluxes of O(1) data exceed the FP16 range (65504) in either
# sweep; the solver's 16-bit cycles scale their residual for the same reason.
SCALE = {"f16": 2.0 ** -6, "bf16": 1.0}


def _kappa(dim, n, kind, seed=700):
    return 1.9 if kind == "const" else synth.kappa_log_uniform(dim, n, seed=seed)


def _dt(name):
    return torch.float16 if name == "f16" else torch.bfloat16


def _rounded(x, name):
    return torch.tensor(x * SCALE[name], dtype=torch.float64).to(_dt(name)).double().numpy()


@pytest.mark.parametrize("name", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", CASES)
def test_mfma_smooth_matches_oracle(dim, n, p, kind, name):
    import paper_2510_00998_amd as hp
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = _rounded(synth.random_vector(nd, seed=71), name)
    b = _rounded(synth.random_rhs(nd, seed=72), name)
    ref = H.smooth(0, u0.copy(), b, 3)
    gm = hp.Solver(dim, n, p, _kappa(dim, n, kind), mfma=1)
    gv = hp.Solver(dim, n, p, _kappa(dim, n, kind))
    um, bd = to_dev(u0, _dt(name)), to_dev(b, _dt(name))
    uv = um.clone()
    gm.smooth(um, bd, 3)
    gv.smooth(uv, bd, 3)
    em, ev = rel_err(to_host(um), ref), rel_err(to_host(uv), ref)
    log(f"mfma smooth {name} dim={dim} n={n} p={p} kappa={kind}: rel err {em:.3e} (vector units {ev:.3e})")
    assert em <= K_SMOOTH * U[name]
    assert not np.array_equal(to_host(um), to_host(uv))  # the matrix-core path ran


@pytest.mark.parametrize("name", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", [(3, 4, 4, "const"), (3, 5, 3, "var"), (3, 3, 5, "const")])
def test_mfma_vcycle_matches_oracle(dim, n, p, kind, name):
    import paper_2510_00998_amd as hp
    H = Hierarchy(dim, n, p, _kappa(dim, n, kind))
    nd = H.fine.ndof
    u0 = _rounded(synth.random_vector(nd, seed=73), name)
    b = _rounded(synth.random_rhs(nd, seed=74), name)
    ref = H.vcycle(0, u0.copy(), b)
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind), mfma=1)
    ud, bd = to_dev(u0, _dt(name)), to_dev(b, _dt(name))
    g.vcycle(ud, bd)
    err = rel_err(to_host(ud), ref)
    log(f"mfma vcycle {name} dim={dim} n={n} p={p} kappa={kind}: rel err {err:.3e}")
    assert err <= K_VCYCLE * U[name]


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dim,n,p,kind", [(3, 6, 4, "const"), (3, 5, 3, "var")])
def test_mfma_cycle_solve_reaches_tolerance(dim, n, p, kind, prec):
    # the FP64 outer iteration restores full accuracy around the
    # matrix-core cycle
    import paper_2510_00998_amd as hp
    s = SIPG(dim, n, p, _kappa(dim, n, kind))
    b = synth.random_rhs(s.ndof, seed=75)
    g = hp.Solver(dim, n, p, _kappa(dim, n, kind), mfma=1,
                  precision=hp.PREC_F16 if prec == "f16" else hp.PREC_BF16)
    xd = torch.zeros(s.ndof, dtype=torch.float64, device="cuda")
    info, st = g.solve(xd, to_dev(b, torch.float64), rtol=1e-10, maxit=300)
    rr = np.linalg.norm(b - s.A @ to_host(xd)) / np.linalg.norm(b)
    log(f"mfma {prec} cycle solve dim={dim} n={n} p={p}: its {info.iterations} oracle residual {rr:.3e}")
    assert st == 0 and rr <= 2e-10
