"""The C++ oracle (oracle/c/sipg_oracle.cpp through oracle/coracle.py) against
what the mathematics fixes and against the pinned NumPy oracle: the same
assembled SIPG operator (paper Section 2.3, eq. weak_form_IP), block-Jacobi
sweeps, V-cycle and MG-preconditioned CG (Section 5), written independently."""
import numpy as np
import pytest

import synth
from oracle import SIPG, Hierarchy
from oracle.coracle import CHierarchy

CASES = [(2, 4, 1, False), (2, 5, 3, True), (3, 3, 2, True), (3, 4, 3, False), (2, 3, 6, False)]


def _kappa(dim, n, var):
    return synth.kappa_log_uniform(dim, n, seed=21) if var else None


@pytest.mark.parametrize("dim,n,p,var", CASES)
def test_matrix_equals_the_numpy_oracle(dim, n, p, var):
    C = CHierarchy(dim, n, p, _kappa(dim, n, var))
    A = SIPG(dim, n, p, _kappa(dim, n, var)).A.tocsr()
    Ac = C.csr()
    assert abs(A - Ac).max() <= 1e-13 * abs(A).max()


@pytest.mark.parametrize("dim,n,p,var", CASES)
def test_smooth_vcycle_solve_equal_the_numpy_oracle(dim, n, p, var):
    kap = _kappa(dim, n, var)
    C = CHierarchy(dim, n, p, kap)
    H = Hierarchy(dim, n, p, kap)
    u = synth.random_vector(C.ndof, seed=3)
    b = synth.random_rhs(C.ndof, seed=4)
    ref = H.smooth(0, u.copy(), b, 3)
    assert np.abs(C.smooth(u, b, 3) - ref).max() <= 1e-12 * np.abs(ref).max()
    ref = H.vcycle(0, u.copy(), b)
    assert np.abs(C.vcycle(u, b) - ref).max() <= 1e-12 * np.abs(ref).max()
    uc, hc = C.solve(b, rtol=1e-10)
    up, hp = H.solve(b, rtol=1e-10)
    assert len(hc) == len(hp) and hc[-1] <= 1e-10 * hc[0]
    assert np.abs(uc - up).max() <= 1e-9 * np.abs(up).max()


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (3, 2, 2)])
def test_symmetric_positive_definite_and_penalty_energy(dim, n, p):
    # invariants on the C++ matrix itself: symmetry, positive definiteness,
    # and a(v, v) of a cell indicator = sigma h^(d-1) (sum over interior
    # facets of kappa_F + 2 kappa_K per boundary facet)
    kap = synth.kappa_log_uniform(dim, n, seed=9)
    A = CHierarchy(dim, n, p, kap).csr().toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)
    nd, h = (p + 1) ** dim, 1.0 / n
    c = n ** dim - 1  # the last cell: upper facets on the boundary
    v = np.zeros(A.shape[0])
    v[c * nd:(c + 1) * nd] = 1.0
    expect = 0.0
    for k in range(dim):
        expect += 2 * kap[c]
        nb = c - n ** k
        expect += 2 * kap[c] * kap[nb] / (kap[c] + kap[nb])
    expect *= 2.0 * (p + 1) ** 2 / h * h ** (dim - 1)
    assert abs(v @ A @ v - expect) <= 1e-12 * expect
