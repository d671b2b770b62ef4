"""hpmg_smooth_noalloc (trace buffers in the library's static device array,
no device allocation) against hpmg_smooth through the C ABI: identical
results on two calls in a row, the second with a smaller input, in every
storage type; sizes beyond the array are rejected."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_common import log, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(hp, dim, n, p, kappa, dtype, nrhs, seed):
    s = hp.Solver(dim, n, p, kappa, max_rhs=nrhs)
    u0 = np.concatenate([synth.random_vector(s.ndof, seed=seed + r) for r in range(nrhs)])
    b = np.concatenate([synth.random_rhs(s.ndof, seed=seed + 10 + r) for r in range(nrhs)])
    return s, u0, b


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
def test_noalloc_smooth_equals_smooth_on_two_calls(dtype):
    import paper_2510_00998_amd as hp
    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    # first call: 3D degree 3, variable kappa, two right-hand sides; second
    # call: a smaller 2D problem with constant kappa and one right-hand side
    cases = [(3, 6, 3, synth.kappa_log_uniform(3, 6, seed=5), 2, 100), (2, 5, 2, 1.3, 1, 200)]
    for dim, n, p, kappa, nrhs, seed in cases:
        s, u0, b = _pair(hp, dim, n, p, kappa, dtype, nrhs, seed)
        ua = to_dev(u0, tdt)
        ub = ua.clone()
        bd = to_dev(b, tdt)
        log(f"noalloc smooth {dtype}: dim={dim} n={n} p={p} nrhs={nrhs}")
        s.smooth(ua, bd, 3, nrhs=nrhs)
        st = s.smooth_noalloc(ub, bd, 3, nrhs=nrhs)
        assert st == 0
        xa, xb = to_host(ua), to_host(ub)
        log(f"  max |diff| {np.abs(xa - xb).max():.3e}")
        assert np.array_equal(xa, xb)
        assert np.abs(xa - u0).max() > 0  # the sweeps did change u


def test_noalloc_rejects_traces_beyond_the_array():
    import paper_2510_00998_amd as hp
    lib = hp.library()
    # Q4 on 32^3 in FP64: 2 x 78.6 MB of traces > 128 MiB
    s = hp.Solver(3, 32, 4, 1.0)
    u = torch.zeros(s.ndof, dtype=torch.float64, device="cuda")
    b = torch.ones(s.ndof, dtype=torch.float64, device="cuda")
    log("noalloc too large: 3D n=32 p=4 FP64")
    st = s.smooth_noalloc(u, b, 1, check=False)
    msg = lib.hpmg_last_error().decode()
    log(f"  status {st}: {msg}")
    assert st == 1 and "static scratch array" in msg
    assert float(torch.abs(u).max()) == 0.0  # nothing ran
    # FP32 fits (2 x 39.3 MB) and matches hpmg_smooth
    u32 = torch.zeros(s.ndof, dtype=torch.float32, device="cuda")
    v32 = torch.zeros_like(u32)
    b32 = b.float()
    assert s.smooth_noalloc(u32, b32, 2) == 0
    s.smooth(v32, b32, 2)
    assert torch.equal(u32, v32)
