"""Rounding floor of the FP64 residual for the log-normal coefficient
workload (degree 5, sigma_log = 2, correlation length 0.1, f = 1), pinned on
a reduced mesh with the same coefficient statistics.

The exact solution u* is approximated in extended precision (x87 long
double, 64-bit significand) by residual refinement around the oracle's
MG-PCG; u64 = fl(u*) is then the best FP64 vector.  Three numbers follow:

* intrinsic floor: the exact residual ||b - A u64|| / ||b|| (long double);
* certified floor: the same residual evaluated in FP64 (what any FP64 solver
  sees at its exit test);
* the a-priori estimate eps ||(|A| |u64|)|| / ||b||, eps = 2^-53.

The FP64 evaluation error of b - A u, not the representability of u, sets
the residual an FP64 solver can certify: the certified floor sits at the
estimate (within a small factor) and above the intrinsic floor.  A solver
whose exit test runs in FP64 therefore stalls near the estimate; at the full
96^3 mesh that estimate is above 1e-10.
"""
import numpy as np

import synth
from oracle import Hierarchy


def _matvec_ld(A, u):
    prod = A.data.astype(np.longdouble) * u.astype(np.longdouble)[A.indices]
    return np.add.reduceat(prod, A.indptr[:-1])


def test_fp64_residual_floor_is_the_evaluation_floor():
    dim, n, p = 3, 3, 5
    kap = synth.kappa_log_normal(dim, n, seed=1005)
    H = Hierarchy(dim, n, p, kap)
    A = H.fine.A.tocsr()
    b = H.fine.load_vector(lambda X: np.ones(X.shape[0]))
    u, hist = H.solve(b, rtol=1e-13, maxit=200)
    ul = u.astype(np.longdouble)
    bl = b.astype(np.longdouble)
    for _ in range(3):
        r = bl - _matvec_ld(A, ul)
        d, _ = H.solve(r.astype(np.float64), rtol=1e-10, maxit=200)
        ul = ul + d.astype(np.longdouble)
    nb = np.linalg.norm(b)
    # the long-double iterate is far more accurate than any FP64 vector
    assert float(np.sqrt(np.sum((bl - _matvec_ld(A, ul)) ** 2))) / nb < 1e-16
    u64 = ul.astype(np.float64)
    rex = bl - _matvec_ld(A, u64)
    intrinsic = float(np.sqrt(np.sum(rex * rex))) / nb
    certified = np.linalg.norm(b - A @ u64) / nb
    est = 2.0 ** -53 * np.linalg.norm(abs(A) @ np.abs(u64)) / nb
    assert 0.2 * est <= certified <= 5.0 * est, (certified, est)
    assert intrinsic < certified, (intrinsic, certified)
    # the FP64 evaluation error of the residual is the certified value itself
    evalerr = np.linalg.norm((b - A @ u64) - rex.astype(np.float64)) / nb
    assert 0.5 * certified <= evalerr <= 1.5 * certified
