"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching a device."""
import ctypes

import pytest

import paper_2510_00998_amd as hp


def test_library_exports_every_declared_symbol():
    lib = hp.library()
    names = hp.declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = hp.library()
    for code in range(7):
        assert lib.hpmg_status_string(code)


def _setup(dim=3, n=4, p=2, per_cell=0, kappa_const=1.0, kappa=None, opt=None):
    lib = hp.library()
    mesh = hp.Mesh(dim, (ctypes.c_int * 3)(n, n, n))
    coeff = hp.Coeff(per_cell, kappa_const, kappa)
    h = ctypes.c_void_p()
    st = lib.hpmg_setup(ctypes.byref(mesh), p, ctypes.byref(coeff), ctypes.byref(opt) if opt else None,
                        None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw", [dict(dim=1), dict(dim=4), dict(n=1), dict(p=0), dict(p=9),
                                dict(kappa_const=0.0), dict(kappa_const=-1.0), dict(kappa_const=float("nan")),
                                dict(per_cell=1, kappa=None)])
def test_setup_rejects_invalid(kw):
    st, h = _setup(**kw)
    assert st == 1, hp.STATUS.get(st)
    assert not h.value
    assert hp.library().hpmg_last_error()


def test_setup_rejects_bad_options():
    for field, val in [("omega_dg", 0.0), ("omega_dg", 1.5), ("omega_cg", -1.0), ("sigma0", 0.0),
                       ("coarsest_n", 1), ("max_rhs", 0), ("precision", 7), ("p_coarsening", 2),
                       ("h_factor", 4), ("h_factor", 1), ("block_recompute", 2),
                       ("block_recompute", 1), ("block_recompute", 2),  # recompute with constant kappa
                       ("block_recompute", 3),
                       ("nu_pre_cg", -2), ("nu_post_cg", -5), ("block_variant", 2), ("mfma", 2)]:
        opt = hp.default_options()
        setattr(opt, field, val)
        st, _ = _setup(opt=opt)
        assert st == 1, field
    # p schedules: not decreasing, below 2, not below p (p = 2 here: any entry)
    for sched in ([3, 3], [1], [2]):
        opt = hp.default_options()
        opt.p_schedule = (ctypes.c_int * 8)(*(sched + [0] * (8 - len(sched))))
        st, _ = _setup(p=4 if sched != [2] else 2, opt=opt)
        assert st == 1, sched
    # interior block with a per-cell kappa, or with no interior cell
    import numpy as np
    k = np.ones(64)
    opt = hp.default_options()
    opt.block_variant = 1
    st, _ = _setup(per_cell=1, kappa=k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), opt=opt)
    assert st == 1
    st, _ = _setup(n=2, opt=opt)
    assert st == 1
    # matrix-core sweeps need dim 3
    opt = hp.default_options()
    opt.mfma = 1
    st, _ = _setup(dim=2, opt=opt)
    assert st == 1
    # an allocator without its free function
    opt = hp.default_options()
    opt.alloc = hp.ALLOC_FN(lambda n, c: None)
    st, _ = _setup(opt=opt)
    assert st == 1


def test_default_options_new_fields():
    o = hp.default_options()
    assert (o.nu_pre, o.nu_post, o.nu_pre_cg, o.nu_post_cg) == (2, 2, -1, -1)
    assert o.block_variant == 0 and list(o.p_schedule) == [0] * 8
    assert not o.alloc and not o.free and not o.alloc_ctx


def test_setup_rejects_nonpositive_per_cell_kappa():
    import numpy as np
    k = np.ones(64)
    k[5] = 0.0
    st, _ = _setup(per_cell=1, kappa=k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert st == 1


def test_null_handle_rejected():
    lib = hp.library()
    assert lib.hpmg_apply_A(None, 0, None, None, 1, None) == 1
    assert lib.hpmg_smooth(None, 0, None, None, 1, 1, None) == 1
    assert lib.hpmg_vcycle(None, 0, None, None, 1, None) == 1
    assert lib.hpmg_solve(None, None, None, 1, 1e-10, 10, None, None) == 1
    assert lib.hpmg_mgmult(None, None, None, 1e-7, 10, 0, None, None) == 1
    assert lib.hpmg_smooth_noalloc(None, 0, None, None, 1, 1, None) == 1
    assert lib.hpmg_ndof(None) == 0
    lib.hpmg_destroy(None)


def test_default_options():
    o = hp.default_options()
    assert o.sigma0 == 2.0 and o.nu_pre == 2 and o.nu_post == 2
    assert abs(o.omega_dg - 0.7) < 1e-15 and abs(o.omega_cg - 2 / 3) < 1e-15


def test_batch_null_arguments_rejected():
    lib = hp.library()
    out = ctypes.c_void_p()
    assert lib.hpmg_batch_create(None, 1, ctypes.byref(out)) == 1
    assert not out.value
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.hpmg_batch_create(arr, 0, ctypes.byref(out)) == 1
    assert lib.hpmg_batch_create(arr, 1, ctypes.byref(out)) == 1  # NULL handle
    assert lib.hpmg_batch_create(arr, 1, None) == 1
    assert lib.hpmg_batch_solve(None, None, None, 1, 1e-10, 10, None, None) == 1
    assert lib.hpmg_batch_tuning(None, None) == 1
    lib.hpmg_batch_destroy(None)
