"""Python binding of libhpmg.so (matrix-free SIPG-DG hp-multigrid on MI355X).

Argument marshalling only: every step of the solver runs in the HIP library.
Vectors are torch tensors on the GPU (float64 or float32, contiguous,
cell-major layout described in include/hpmg.h); work is enqueued on the
current torch stream.  Importing this package fails loudly if the library
has not been built (python paper_2510_00998_amd/csrc/build.py).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhpmg.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "hpmg.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libhpmg.so not built at {LIB_PATH}; run `python paper_2510_00998_amd/csrc/build.py`")
# The tensors and streams handed to the library belong to torch's HIP runtime.
# Loading torch first makes the library's libamdhip64.so.7 dependency resolve
# to that same, already loaded runtime (one runtime per process); loaded the
# other way round, the process would hold two HIP runtimes side by side.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "HPMG_OK", 1: "HPMG_E_INVALID", 2: "HPMG_E_NOMEM", 3: "HPMG_E_DEVICE",
          4: "HPMG_E_NOT_CONVERGED", 5: "HPMG_E_BREAKDOWN", 6: "HPMG_E_UNSUPPORTED"}
F64, F32, F16, BF16 = 0, 1, 2, 3
PREC_F64, PREC_F32, PREC_F16, PREC_BF16 = 0, 1, 2, 3


def _torch_dtype(code):
    import torch
    return {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[code]


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3)]


class AdaptiveMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("refine", ctypes.c_int), ("nleaf", ctypes.c_int),
                ("leaves", ctypes.POINTER(ctypes.c_int))]


class Coeff(ctypes.Structure):
    _fields_ = [("per_cell", ctypes.c_int), ("kappa_const", ctypes.c_double),
                ("kappa", ctypes.POINTER(ctypes.c_double))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("sigma0", ctypes.c_double), ("omega_dg", ctypes.c_double), ("omega_cg", ctypes.c_double),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("coarsest_n", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_rhs", ctypes.c_int), ("p_coarsening", ctypes.c_int),
                ("h_factor", ctypes.c_int), ("basis", ctypes.c_int), ("block_recompute", ctypes.c_int),
                ("nu_pre_cg", ctypes.c_int), ("nu_post_cg", ctypes.c_int), ("block_variant", ctypes.c_int),
                ("p_schedule", ctypes.c_int * 8), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("mfma", ctypes.c_int), ("spacetree_levels", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("initial_residual", ctypes.c_double),
                ("final_residual", ctypes.c_double), ("residual_history", ctypes.c_double * 256),
                ("seconds", ctypes.c_double)]


_vp = ctypes.c_void_p
_lib.hpmg_default_options.argtypes = [ctypes.POINTER(Options)]
_lib.hpmg_default_options.restype = None
_lib.hpmg_setup.argtypes = [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.POINTER(Coeff), ctypes.POINTER(Options),
                            _vp, ctypes.POINTER(_vp)]
_lib.hpmg_setup.restype = ctypes.c_int
_lib.hpmg_setup_adaptive.argtypes = [ctypes.POINTER(AdaptiveMesh), ctypes.c_int, ctypes.POINTER(Coeff),
                                     ctypes.POINTER(Options), _vp, ctypes.POINTER(_vp)]
_lib.hpmg_setup_adaptive.restype = ctypes.c_int
_lib.hpmg_ndof.argtypes = [_vp]
_lib.hpmg_ndof.restype = ctypes.c_size_t
_lib.hpmg_load_vector.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _vp]
_lib.hpmg_load_vector.restype = ctypes.c_int
_lib.hpmg_apply_A.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp]
_lib.hpmg_apply_A.restype = ctypes.c_int
_lib.hpmg_smooth.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
_lib.hpmg_smooth.restype = ctypes.c_int
_lib.hpmg_smooth_noalloc.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
_lib.hpmg_smooth_noalloc.restype = ctypes.c_int
_lib.hpmg_project.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp]
_lib.hpmg_project.restype = ctypes.c_int
_lib.hpmg_sweep.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
_lib.hpmg_sweep.restype = ctypes.c_int
_lib.hpmg_vcycle.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp]
_lib.hpmg_vcycle.restype = ctypes.c_int
_lib.hpmg_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                            ctypes.POINTER(SolveInfo), _vp]
_lib.hpmg_solve.restype = ctypes.c_int
_lib.hpmg_mgmult.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(SolveInfo), _vp]
_lib.hpmg_mgmult.restype = ctypes.c_int
_lib.hpmg_destroy.argtypes = [_vp]
_lib.hpmg_destroy.restype = None
_lib.hpmg_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)]
_lib.hpmg_batch_create.restype = ctypes.c_int
_lib.hpmg_batch_solve.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.POINTER(SolveInfo), _vp]
_lib.hpmg_batch_solve.restype = ctypes.c_int
_lib.hpmg_batch_smooth.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int,
                                   ctypes.c_int, _vp]
_lib.hpmg_batch_smooth.restype = ctypes.c_int
_lib.hpmg_batch_tuning.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_lib.hpmg_batch_tuning.restype = ctypes.c_int
_lib.hpmg_batch_set_tuning.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_lib.hpmg_batch_set_tuning.restype = ctypes.c_int
_lib.hpmg_batch_destroy.argtypes = [_vp]
_lib.hpmg_batch_destroy.restype = None
_lib.hpmg_status_string.argtypes = [ctypes.c_int]
_lib.hpmg_status_string.restype = ctypes.c_char_p
_lib.hpmg_last_error.argtypes = []
_lib.hpmg_last_error.restype = ctypes.c_char_p


class HpmgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.hpmg_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(st: int, where: str):
    if st != 0:
        raise HpmgError(st, where)


def library():
    """The loaded ctypes library (for ABI tests)."""
    return _lib


def declared_symbols() -> list[str]:
    """Names of the functions declared in include/hpmg.h."""
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(hpmg_[a-z_A]+)\s*\(", txt)))


def default_options() -> Options:
    o = Options()
    _lib.hpmg_default_options(ctypes.byref(o))
    return o


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype_code=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype_code is not None:
        want = _torch_dtype(dtype_code)
        if t.dtype != want:
            raise TypeError(f"expected {want}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _code(t):
    import torch
    codes = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return codes[t.dtype]


class Solver:
    """One SIPG problem -div(kappa grad u) = f on [0,1]^dim (hpmg_setup, or
    hpmg_setup_adaptive when `leaves` is given)."""

    def __init__(self, dim: int, n: int, p: int, kappa=1.0, stream=None, allocator=None, leaves=None,
                 refine: int = 2, **options):
        """options: fields of hpmg_options (p_schedule as a sequence of degrees);
        allocator: optional (alloc(nbytes) -> device pointer int, free(pointer))
        pair through which the library obtains every device buffer of the
        handle (e.g. torch's caching allocator); kept alive with the solver;
        leaves: (nleaf, 1 + dim) integer rows (level, coordinates) of an
        adaptive mesh over n^dim base cells with subdivision factor refine."""
        opt = default_options()
        for k, v in options.items():
            if not hasattr(opt, k) or k in ("alloc", "free", "alloc_ctx"):
                raise KeyError(f"unknown option {k}")
            if k == "p_schedule":
                sched = list(v) + [0] * (8 - len(v))
                if len(sched) > 8:
                    raise ValueError("p_schedule holds at most 7 degrees")
                opt.p_schedule = (ctypes.c_int * 8)(*sched)
            else:
                setattr(opt, k, v)
        self._alloc_cbs = None
        if allocator is not None:
            fa, ff = allocator

            def _a(nbytes, _ctx):
                try:
                    return int(fa(int(nbytes)))
                except Exception:
                    return None

            def _f(ptr, _ctx):
                ff(int(ptr))

            self._alloc_cbs = (ALLOC_FN(_a), FREE_FN(_f))
            opt.alloc, opt.free = self._alloc_cbs
        mesh = Mesh(dim, (ctypes.c_int * 3)(n, n, n))
        self._kappa_buf = None
        if np.isscalar(kappa):
            coeff = Coeff(0, float(kappa), None)
        else:
            arr = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64))
            if arr.shape != (n ** dim,):
                raise ValueError("kappa must hold one value per cell")
            self._kappa_buf = arr
            coeff = Coeff(1, 0.0, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        self.leaves = None
        if leaves is not None:
            lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32))
            if lv.ndim != 2 or lv.shape[1] != 1 + dim:
                raise ValueError("leaves must have shape (nleaf, 1 + dim)")
            self.leaves = lv
            am = AdaptiveMesh(dim, n, refine, lv.shape[0], lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
            _check(_lib.hpmg_setup_adaptive(ctypes.byref(am), p, ctypes.byref(coeff), ctypes.byref(opt),
                                            _stream(stream), ctypes.byref(h)), "hpmg_setup_adaptive")
        else:
            _check(_lib.hpmg_setup(ctypes.byref(mesh), p, ctypes.byref(coeff), ctypes.byref(opt), _stream(stream),
                                   ctypes.byref(h)), "hpmg_setup")
        self._h = h
        self.dim, self.n, self.p, self.options = dim, n, p, opt
        self.ndof = int(_lib.hpmg_ndof(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.hpmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_vector(self, kind: int, param: float, b, stream=None):
        """kind 0: f = param; 1: f = -Laplace prod sin(param pi x_i); 2 (2D): the two-peak f."""
        prm = (ctypes.c_double * 1)(param)
        _check(_lib.hpmg_load_vector(self._h, kind, prm, _ptr(b, F64), _stream(stream)), "hpmg_load_vector")
        return b

    def apply_A(self, u, y, nrhs: int = 1, stream=None):
        c = _code(u)
        _check(_lib.hpmg_apply_A(self._h, c, _ptr(u, c), _ptr(y, c), nrhs, _stream(stream)), "hpmg_apply_A")
        return y

    def smooth(self, u, b, nsweeps: int, nrhs: int = 1, stream=None):
        c = _code(u)
        _check(_lib.hpmg_smooth(self._h, c, _ptr(u, c), _ptr(b, c), nsweeps, nrhs, _stream(stream)), "hpmg_smooth")
        return u

    def smooth_noalloc(self, u, b, nsweeps: int, nrhs: int = 1, stream=None, check=True):
        """hpmg_smooth_noalloc: hpmg_smooth with the traces in the static scratch array."""
        c = _code(u)
        st = _lib.hpmg_smooth_noalloc(self._h, c, _ptr(u, c), _ptr(b, c), nsweeps, nrhs, _stream(stream))
        if check:
            _check(st, "hpmg_smooth_noalloc")
        return st

    def project(self, u, nrhs: int = 1, stream=None):
        c = _code(u)
        _check(_lib.hpmg_project(self._h, c, _ptr(u, c), nrhs, _stream(stream)), "hpmg_project")
        return u

    def sweep(self, u, b, nsweeps: int = 1, nrhs: int = 1, stream=None):
        c = _code(u)
        _check(_lib.hpmg_sweep(self._h, c, _ptr(u, c), _ptr(b, c), nsweeps, nrhs, _stream(stream)), "hpmg_sweep")
        return u

    def vcycle(self, u, b, nrhs: int = 1, stream=None):
        c = _code(u)
        _check(_lib.hpmg_vcycle(self._h, c, _ptr(u, c), _ptr(b, c), nrhs, _stream(stream)), "hpmg_vcycle")
        return u

    def mgmult(self, u, b, rtol: float = 1e-7, maxit: int = 500, exit: str = "unprec", stream=None, check=True):
        """Stationary multigrid iteration (hpmg_mgmult); exit "unprec" or "prec"."""
        info = SolveInfo()
        st = _lib.hpmg_mgmult(self._h, _ptr(u, F64), _ptr(b, F64), rtol, maxit, 0 if exit == "unprec" else 1,
                              ctypes.byref(info), _stream(stream))
        if check:
            _check(st, "hpmg_mgmult")
        return info, st

    def solve(self, u, b, rtol: float = 1e-10, maxit: int = 200, nrhs: int = 1, stream=None, check=True):
        info = SolveInfo()
        st = _lib.hpmg_solve(self._h, _ptr(u, F64), _ptr(b, F64), nrhs, rtol, maxit, ctypes.byref(info),
                             _stream(stream))
        if check:
            _check(st, "hpmg_solve")
        return info, st


class Batch:
    """Independent problems solved together (hpmg_batch_create / hpmg_batch_solve).

    The solvers must stay alive while the batch is used; keep references."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (_vp * len(self.solvers))(*[s._h for s in self.solvers])
        b = _vp()
        _check(_lib.hpmg_batch_create(arr, len(self.solvers), ctypes.byref(b)), "hpmg_batch_create")
        self._b = b

    def close(self):
        if getattr(self, "_b", None):
            _lib.hpmg_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tuning(self) -> dict:
        """Autotuned launch configuration (hpmg_batch_tuning)."""
        out = (ctypes.c_int * 9)()
        _check(_lib.hpmg_batch_tuning(self._b, out), "hpmg_batch_tuning")

        def half_tiles(mask):  # degrees p whose launches use half the cells per workgroup
            return [n - 1 for n in range(2, 31) if (mask >> n) & 1]
        return {"vcycle_grid": out[0], "vcycle_split_by_degree": bool(out[1]),
                "smooth_f32_grid": out[2], "smooth_f32_split_by_degree": bool(out[3]),
                "smooth_f64_grid": out[4], "smooth_f64_split_by_degree": bool(out[5]),
                "vcycle_half_tile_degrees": half_tiles(out[6]),
                "smooth_f32_half_tile_degrees": half_tiles(out[7]),
                "smooth_f64_half_tile_degrees": half_tiles(out[8])}

    def set_tuning(self, cfg):
        """Replace the launch configuration (hpmg_batch_set_tuning): cfg is the
        9-int list of hpmg_batch_tuning (see tuning_raw)."""
        arr = (ctypes.c_int * 9)(*cfg)
        _check(_lib.hpmg_batch_set_tuning(self._b, arr), "hpmg_batch_set_tuning")

    @property
    def tuning_raw(self) -> list:
        out = (ctypes.c_int * 9)()
        _check(_lib.hpmg_batch_tuning(self._b, out), "hpmg_batch_tuning")
        return list(out)

    @property
    def grid(self) -> int:
        return self.tuning["vcycle_grid"]

    def smooth(self, us, bs, nsweeps: int, nrhs: int = 1, stream=None):
        """Projection plus nsweeps fused sweeps of every problem (FP64 or FP32 tensors)."""
        m = len(self.solvers)
        if len(us) != m or len(bs) != m:
            raise ValueError("one u and one b per problem")
        c = _code(us[0])
        for s, u, b in zip(self.solvers, us, bs):
            if u.numel() != nrhs * s.ndof or b.numel() != nrhs * s.ndof:
                raise ValueError("vector size must be nrhs * ndof")
        up = (_vp * m)(*[_ptr(u, c) for u in us])
        bp = (_vp * m)(*[_ptr(b, c) for b in bs])
        _check(_lib.hpmg_batch_smooth(self._b, c, up, bp, nsweeps, nrhs, _stream(stream)), "hpmg_batch_smooth")

    def solve(self, us, bs, rtol: float = 1e-10, maxit: int = 200, nrhs: int = 1, stream=None, check=True):
        """us[j], bs[j]: FP64 device tensors of nrhs * ndof_j values. Returns (infos, status)."""
        m = len(self.solvers)
        if len(us) != m or len(bs) != m:
            raise ValueError("one u and one b per problem")
        for s, u, b in zip(self.solvers, us, bs):
            if u.numel() != nrhs * s.ndof or b.numel() != nrhs * s.ndof:
                raise ValueError("vector size must be nrhs * ndof")
        up = (_vp * m)(*[_ptr(u, F64) for u in us])
        bp = (_vp * m)(*[_ptr(b, F64) for b in bs])
        infos = (SolveInfo * m)()
        st = _lib.hpmg_batch_solve(self._b, up, bp, nrhs, rtol, maxit, infos, _stream(stream))
        if check:
            _check(st, "hpmg_batch_solve")
        return list(infos), st
