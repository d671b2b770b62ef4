"""Pins of the oracle's assembled SIPG operator (paper Section 2.3,
eq. weak_form_IP with theta = -1, harmonic face coefficient, penalty
gamma_F = sigma interior / 2 sigma boundary) against what mathematics fixes."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

import synth
from oracle import SIPG, manufactured as mf


def _dense(s):
    return s.A.toarray()


@pytest.mark.parametrize("dim,n,p", [(2, 3, 1), (2, 4, 2), (2, 3, 4), (3, 2, 1), (3, 3, 2), (3, 2, 3)])
@pytest.mark.parametrize("varkappa", [False, True])
def test_symmetric_positive_definite(dim, n, p, varkappa):
    kappa = synth.kappa_log_uniform(dim, n, seed=7) if varkappa else None
    A = _dense(SIPG(dim, n, p, kappa))
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)  # raises if not positive definite


@pytest.mark.parametrize("dim,n,p", [(2, 4, 1), (2, 4, 3), (3, 3, 2)])
def test_global_linear_annihilated_away_from_boundary(dim, n, p):
    # (A l)_i = -int_K div(grad l) phi_i = 0 for rows of cells not touching
    # the boundary: jumps of l vanish and its normal flux is single-valued.
    s = SIPG(dim, n, p)
    X = s.dof_coords()
    coef = np.array([2.0, -3.0, 0.5])[:dim]
    ell = 1.0 + X @ coef
    y = (s.A @ ell).reshape(s.ncell, s.nd)
    cc = s.cell_index_coords()
    interior = np.all((cc > 0) & (cc < n - 1), axis=1)
    assert interior.any()
    assert np.abs(y[interior]).max() < 1e-11 * np.abs(s.A.data).max()
    assert np.abs(y[~interior]).max() > 1e-3  # boundary rows see the Dirichlet terms


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (3, 2, 1), (3, 2, 3)])
def test_penalty_energy_of_cell_indicator(dim, n, p):
    # u = 1 on one cell, 0 elsewhere: only penalty terms survive,
    # a(u,u) = sigma h^(d-1) [sum_interior kappa_F + 2 sum_boundary kappa_K].
    kappa = synth.kappa_log_uniform(dim, n, seed=11)
    s = SIPG(dim, n, p, kappa)
    c = 0
    u = np.zeros(s.ndof)
    u[c * s.nd:(c + 1) * s.nd] = 1.0
    energy = u @ (s.A @ u)
    cc = s.cell_index_coords()[c]
    expect = 0.0
    for k in range(dim):
        for side in (0, 1):
            at_bdy = cc[k] == (0 if side == 0 else n - 1)
            if at_bdy:
                expect += 2 * kappa[c]
            else:
                nb = c + (n ** k if side == 1 else -n ** k)
                expect += 2 * kappa[c] * kappa[nb] / (kappa[c] + kappa[nb])
    sigma = 2.0 * (p + 1) ** 2 / s.h
    expect *= sigma * s.h ** (dim - 1)
    assert abs(energy - expect) < 1e-12 * expect


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (2, 4, 3), (3, 2, 2), (3, 3, 2), (3, 2, 4)])
def test_polynomial_solution_reproduced(dim, n, p):
    # Galerkin consistency: u = prod x_i(1-x_i) lies in Q_p (p >= 2) and is the
    # exact solution, so the discrete solution is its interpolant.
    u, f = mf.bubble(dim)
    s = SIPG(dim, n, p, kappa=3.0)
    b = 3.0 * s.load_vector(f)
    x = spla.spsolve(s.A.tocsc(), b)
    assert np.abs(x - s.interpolate(u)).max() < 1e-12


def _layered_solution(dim, k1, k2, beta):
    """Piecewise-quadratic solution of -div(k grad u) = f with k = k1 for
    x < 1/2, k2 for x > 1/2: continuous u and continuous flux k du/dx."""
    X = sy.symbols("x0:3", real=True)[:dim]
    A = (k1 + k2 * (1 + beta) / 2) / (k1 + k2)
    C = A - sy.Rational(1, 2) + beta / 2
    x = X[0]
    rest = sy.Mul(*[t * (1 - t) for t in X[1:]])
    left = (A * x - x ** 2) * rest
    right = (C * (1 - x) - beta * (1 - x) ** 2) * rest
    fl = -k1 * sum(sy.diff(left, t, 2) for t in X)
    fr = -k2 * sum(sy.diff(right, t, 2) for t in X)
    ul, ur = sy.lambdify(X, left), sy.lambdify(X, right)
    fl, fr = sy.lambdify(X, fl), sy.lambdify(X, fr)

    def u(P):
        a = [P[:, k] for k in range(dim)]
        return np.where(P[:, 0] <= 0.5, ul(*a) + 0 * P[:, 0], ur(*a) + 0 * P[:, 0])

    def f(P):
        a = [P[:, k] for k in range(dim)]
        return np.where(P[:, 0] < 0.5, fl(*a) + 0 * P[:, 0], fr(*a) + 0 * P[:, 0])
    return u, f


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (2, 2, 3), (3, 2, 2)])
def test_layered_coefficient_solution_reproduced(dim, n, p):
    # SWIP consistency with the harmonic face coefficient: a piecewise
    # polynomial solution with continuous flux is reproduced exactly.
    k1, k2 = 1.0, 10.0
    u, f = _layered_solution(dim, k1, k2, sy.Rational(1, 2))
    s0 = SIPG(dim, n, p)
    xc = s0.cell_index_coords()[:, 0]
    kappa = np.where(xc < n // 2, k1, k2)
    s = SIPG(dim, n, p, kappa)
    b = s.load_vector(f)
    x = spla.spsolve(s.A.tocsc(), b)
    assert np.abs(x - s.interpolate(u)).max() < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("which", ["sin", "two_peak"])
def test_manufactured_convergence_rate(p, which):
    # Section 6.1: the error decreases like h^(p+1)
    u, f = mf.sin_product(2, 2) if which == "sin" else mf.two_peak()
    ns = [8, 16, 32] if which == "two_peak" else [4, 8, 16]
    errs = []
    for n in ns:
        s = SIPG(2, n, p)
        x = spla.spsolve(s.A.tocsc(), s.load_vector(f))
        errs.append(s.l2_error(x, u))
    rate = np.log2(errs[-2] / errs[-1])
    assert abs(rate - (p + 1)) < 0.25, (errs, rate)


def test_manufactured_convergence_rate_3d():
    u, f = mf.sin_product(3, 1)
    errs = []
    for n in [2, 4, 8]:
        s = SIPG(3, n, 2)
        x = spla.spsolve(s.A.tocsc(), s.load_vector(f))
        errs.append(s.l2_error(x, u))
    rate = np.log2(errs[-2] / errs[-1])
    assert abs(rate - 3) < 0.25, (errs, rate)


@pytest.mark.parametrize("dim,n,p", [(2, 5, 2), (3, 4, 2)])
def test_block_rows_match_assembled(dim, n, p):
    kappa = synth.kappa_log_uniform(dim, n, seed=3)
    s = SIPG(dim, n, p, kappa)
    u = synth.random_vector(s.ndof, seed=5)
    cells = np.array([0, 1, s.ncell // 2, s.ncell - 1])
    y = (s.A @ u).reshape(s.ncell, s.nd)
    assert np.allclose(s.apply_rows(cells, u), y[cells], rtol=0, atol=1e-12 * np.abs(y).max())


def _to_nodes(s_from, u, nodes_to):
    """Nodal values of the DG function u (basis of s_from) at other nodes, per cell."""
    from oracle.basis import lagrange_1d
    from oracle.sipg import _kron_dims
    E, _ = lagrange_1d(s_from.nodes1d, nodes_to)
    T = _kron_dims([E] * s_from.dim)
    return (u.reshape(s_from.ncell, -1) @ T.T).ravel()


@pytest.mark.parametrize("dim,n,p,varkappa", [(2, 4, 3, False), (2, 3, 4, True), (3, 2, 2, True)])
def test_gauss_legendre_basis_gives_the_same_discrete_solution(dim, n, p, varkappa):
    # Gauss-Lobatto and Gauss-Legendre nodes span the same Q_p space and the
    # bilinear form does not depend on the basis: the Galerkin solutions are
    # the same function (Section 4.1 remark on the two node families)
    kappa = synth.kappa_log_uniform(dim, n, seed=17) if varkappa else None
    _, f = mf.sin_product(dim, 1)
    s1 = SIPG(dim, n, p, kappa, basis="gll")
    s2 = SIPG(dim, n, p, kappa, basis="gl")
    u1 = spla.spsolve(s1.A.tocsc(), s1.load_vector(f))
    u2 = spla.spsolve(s2.A.tocsc(), s2.load_vector(f))
    u1_at_gl = _to_nodes(s1, u1, s2.nodes1d)
    assert np.abs(u1_at_gl - u2).max() <= 1e-11 * np.abs(u2).max()
    A2 = s2.A.toarray()
    assert np.abs(A2 - A2.T).max() <= 1e-14 * np.abs(A2).max()
    np.linalg.cholesky(A2)


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (3, 2, 3)])
def test_gauss_legendre_mass_is_diagonal_and_bubble_reproduced(dim, n, p):
    from oracle.basis import gl_nodes, ref_matrices_1d
    M, _ = ref_matrices_1d(p, gl_nodes(p))
    assert np.abs(M - np.diag(np.diag(M))).max() <= 1e-15
    u, f = mf.bubble(dim)
    s = SIPG(dim, n, p, basis="gl")
    uh = spla.spsolve(s.A.tocsc(), s.load_vector(f))
    assert np.abs(uh - s.interpolate(u)).max() <= 1e-11
