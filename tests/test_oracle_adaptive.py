"""Pins of the oracle's SIPG operator and hp-multigrid on adaptive spacetree
meshes (paper Section 2.1, hierarchical Cartesian meshes; Section 2.3, eq.
weak_form_IP on their leaves) against what mathematics and the pinned
uniform-mesh oracle fix."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import SIPG, q1_stiffness
from oracle.adaptive import AdaptiveHierarchy, AdaptiveSIPG
from oracle.mg import HierarchyOptions


def _mesh(dim, n, r, kind="ball", max_level=1, seed=3):
    if kind == "ball":
        ref = synth.ball_refinement([(0.3, 0.4, 0.45)], [0.2])
    else:
        ref = synth.random_refinement(seed, 0.35)
    return synth.spacetree_leaves(dim, n, r, ref, max_level)


def _has_hanging(s):
    return any(h < min(s.h[a], s.h[b]) - 1e-15 or s.h[a] != s.h[b] for a, b, _, side, h, _ in s.pieces
               if side == 0)


@pytest.mark.parametrize("dim,n,r,p", [(2, 3, 2, 2), (2, 2, 3, 1), (3, 2, 2, 2)])
def test_one_level_meshes_equal_the_uniform_oracle(dim, n, r, p):
    # all leaves on level 0: the uniform n^d mesh; all leaves on level 1: the
    # uniform (n r)^d mesh with the cells in depth-first order
    base = synth.spacetree_leaves(dim, n, r, lambda *a: False, 0)
    A0 = AdaptiveSIPG(dim, n, r, base, p).A.toarray()
    U0 = SIPG(dim, n, p).A.toarray()
    assert np.abs(A0 - U0).max() <= 1e-12 * np.abs(U0).max()
    fine = synth.spacetree_leaves(dim, n, r, lambda *a: True, 1)
    s = AdaptiveSIPG(dim, n, r, fine, p)
    u = SIPG(dim, n * r, p)
    m = n * r
    cid = sum(fine[:, 1 + k] * m ** k for k in range(dim))
    perm = (cid[:, None] * s.nd + np.arange(s.nd)[None, :]).ravel()
    Uf = u.A.toarray()[np.ix_(perm, perm)]
    assert np.abs(s.A.toarray() - Uf).max() <= 1e-12 * np.abs(Uf).max()


@pytest.mark.parametrize("dim,n,r,p,kind", [(2, 3, 2, 1, "ball"), (2, 3, 2, 3, "random"), (2, 2, 3, 2, "ball"),
                                            (3, 2, 2, 1, "ball"), (3, 2, 2, 2, "random"), (3, 2, 3, 1, "ball")])
def test_symmetric_positive_definite_with_hanging_facets(dim, n, r, p, kind):
    s = AdaptiveSIPG(dim, n, r, _mesh(dim, n, r, kind), p)
    assert _has_hanging(s)
    A = s.A.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)


@pytest.mark.parametrize("dim,n,r,p,lev", [(2, 2, 2, 2, 2), (2, 3, 3, 3, 1), (2, 2, 2, 4, 1), (3, 2, 2, 2, 1),
                                           (3, 2, 3, 2, 1)])
def test_polynomial_solution_reproduced_across_hanging_facets(dim, n, r, p, lev):
    # u = prod x_i(1-x_i) lies in Q_p (p >= 2) on every leaf and vanishes on
    # the boundary: by consistency of the form, the discrete solution is its
    # interpolant, which needs every hanging-facet integral exact
    s = AdaptiveSIPG(dim, n, r, _mesh(dim, n, r, max_level=lev), p)
    assert _has_hanging(s)

    def u(X):
        return np.prod(X * (1 - X), axis=1)

    def f(X):
        q = X * (1 - X)
        return sum(2.0 * np.prod(np.delete(q, i, axis=1), axis=1) for i in range(dim))

    uh = spla.spsolve(s.A.tocsc(), s.load_vector(f))
    ui = s.interpolate(u)
    assert np.abs(uh - ui).max() <= 1e-10 * np.abs(ui).max()


@pytest.mark.parametrize("dim,n,r,p", [(2, 4, 2, 1), (2, 4, 3, 2), (3, 3, 2, 2)])
def test_global_linear_annihilated_away_from_boundary(dim, n, r, p):
    s = AdaptiveSIPG(dim, n, r, _mesh(dim, n, r), p)
    X = s.dof_coords()
    ell = 1.0 + X @ np.array([2.0, -3.0, 0.5])[:dim]
    y = (s.A @ ell).reshape(s.ncell, s.nd)
    lo, hi = s.origin, s.origin + s.h[:, None]
    interior = np.all((lo > 1e-12) & (hi < 1 - 1e-12), axis=1)
    assert interior.any() and _has_hanging(s)
    assert np.abs(y[interior]).max() < 1e-11 * np.abs(s.A.data).max()


@pytest.mark.parametrize("dim,n,r,p", [(2, 3, 2, 2), (2, 2, 3, 3), (3, 2, 2, 1)])
def test_penalty_energy_of_leaf_indicators(dim, n, r, p):
    # v = 1 on one leaf: only penalty terms survive, a(v, v) = sum over the
    # leaf's facet pieces of sigma |piece| (sigma = sigma0 (p+1)^2 / width of
    # the finer side) plus 2 sigma0 (p+1)^2 / h |facet| on the boundary;
    # pieces counted from the geometry of the leaves, not from the oracle
    leaves = _mesh(dim, n, r)
    s = AdaptiveSIPG(dim, n, r, leaves, p)
    pen = 2.0 * (p + 1) ** 2
    lo, h = s.origin, s.h
    for K in range(s.ncell):
        v = np.zeros(s.ndof)
        v[K * s.nd:(K + 1) * s.nd] = 1.0
        expect = 0.0
        for k in range(dim):
            for side in (0, 1):
                x = lo[K, k] + side * h[K]
                if x < 1e-12 or x > 1 - 1e-12:
                    expect += 2 * pen / h[K] * h[K] ** (dim - 1)
                    continue
                # leaves touching this facet from the other side
                for J in range(s.ncell):
                    y = lo[J, k] + (1 - side) * h[J]
                    if abs(y - x) > 1e-12:
                        continue
                    ov = 1.0
                    for t in range(dim):
                        if t != k:
                            ov *= max(0.0, min(lo[K, t] + h[K], lo[J, t] + h[J]) - max(lo[K, t], lo[J, t]))
                    if ov > 0:
                        expect += pen / min(h[K], h[J]) * ov
        assert abs(v @ (s.A @ v) - expect) <= 1e-12 * expect


@pytest.mark.parametrize("dim,n,r", [(2, 4, 2), (2, 3, 3), (3, 3, 2)])
def test_base_q1_galerkin_product_is_q1_stiffness(dim, n, r):
    # the base mesh's continuous Q1 functions are in every DG_p space on the
    # leaves; for them the jumps vanish, so P^T A P is their Q1 stiffness
    s = AdaptiveSIPG(dim, n, r, _mesh(dim, n, r), 2)
    P = s.base_q1_prolongation()
    G = (P.T @ s.A @ P).toarray()
    Q = q1_stiffness(dim, n).toarray()
    assert np.abs(G - Q).max() <= 1e-12 * np.abs(Q).max()


@pytest.mark.parametrize("dim,n,r,p,sched", [(2, 4, 2, 4, "halve"), (2, 3, 3, 3, "direct"), (3, 2, 2, 3, "halve")])
def test_mg_pcg_equals_direct_solve(dim, n, r, p, sched):
    leaves = _mesh(dim, n, r, "random")
    H = AdaptiveHierarchy(dim, n, r, leaves, p, HierarchyOptions(p_coarsening=sched, coarsest_n=2))
    A = H.levels[0].A
    b = synth.random_rhs(A.shape[0], seed=5)
    u, hist = H.solve(b, rtol=1e-11, maxit=200)
    ud = spla.spsolve(A.tocsc(), b)
    assert hist[-1] <= 1e-11 * hist[0]
    assert np.abs(u - ud).max() <= 1e-8 * np.abs(ud).max()
    assert len(hist) < 150


@pytest.mark.parametrize("p", [2, 3])
def test_manufactured_convergence_rate_on_adaptive_meshes(p):
    # u = sin(pi x) sin(pi y), the same refinement region on base meshes
    # 8, 16, 32: the L2 error falls as h^(p+1)
    def u(X):
        return np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])

    def f(X):
        return 2 * np.pi ** 2 * u(X)

    errs = []
    for n in (8, 16, 32):
        leaves = synth.spacetree_leaves(2, n, 2, synth.ball_refinement([(0.3, 0.4)], [0.2]), 1)
        s = AdaptiveSIPG(2, n, 2, leaves, p)
        uh = spla.spsolve(s.A.tocsc(), s.load_vector(f))
        errs.append(s.l2_error(uh, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - (p + 1)) < 0.3), rates


def test_rejects_unbalanced_and_overlapping_leaves():
    leaves = synth.spacetree_leaves(2, 2, 2, lambda *a: False, 0)
    bad = np.vstack([leaves, [[1, 0, 0]]])
    with pytest.raises(ValueError):
        AdaptiveSIPG(2, 2, 2, bad, 1)
    # a level-2 leaf next to a level-0 leaf
    raw = []
    for row in leaves:
        if row[1] == 0 and row[2] == 0:
            for m in range(4):
                cx, cy = m % 2, m // 2
                if m == 3:
                    for q in range(4):
                        raw.append([2, 2 * cx + q % 2, 2 * cy + q // 2])
                else:
                    raw.append([1, cx, cy])
        else:
            raw.append(list(row))
    with pytest.raises(ValueError):
        AdaptiveSIPG(2, 2, 2, np.array(raw), 1)


def test_row_blocks_equal_the_assembled_rows():
    leaves = _mesh(3, 2, 2, "random")
    s = AdaptiveSIPG(3, 2, 2, leaves, 2, kappa=1.7)
    A = s.A.toarray()
    cells = [0, 5, len(leaves) - 1]
    rb = s.row_blocks(cells)
    nd = s.nd
    for K in cells:
        row = np.zeros((nd, s.ndof))
        for J, B in rb[K].items():
            row[:, J * nd:(J + 1) * nd] = B
        assert np.abs(row - A[K * nd:(K + 1) * nd]).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("dim,n,r,lev", [(2, 4, 2, 2), (2, 3, 3, 1), (3, 2, 2, 2)])
def test_spacetree_levels_are_balanced_meshes_and_transfers_reproduce_polynomials(dim, n, r, lev):
    # one level up at a time: every coarser leaf set is a valid balanced
    # mesh, the last one is the base mesh, and the transfer maps the coarse
    # interpolant of a global polynomial of the level's degree to the fine one
    from oracle.adaptive import coarser_leaves, spacetree_prolongation
    lv = _mesh(dim, n, r, "random", max_level=lev)
    q = 2
    coef = np.array([0.7, -1.3, 0.4])[:dim]

    def poly(X):  # in Q_2: degree <= 2 in every coordinate
        return (X @ coef + 0.5) ** 2 - X[:, 0] * X[:, -1]

    while lv[:, 0].max() > 0:
        lc, parent = coarser_leaves(lv, r)
        fine = AdaptiveSIPG(dim, n, r, lv, q)
        coarse = AdaptiveSIPG(dim, n, r, lc, q)  # validates coverage and balance
        P = spacetree_prolongation(fine, coarse, parent)
        assert np.abs(P @ coarse.interpolate(poly) - fine.interpolate(poly)).max() <= 1e-12
        assert lc[:, 0].max() == lv[:, 0].max() - 1
        lv = lc
    assert len(lv) == n ** dim


def test_spacetree_levels_cut_the_iteration_count():
    leaves = synth.spacetree_leaves(2, 8, 2, synth.ball_refinement([(0.3, 0.4)], [0.2]), 2)
    b = synth.random_rhs(len(leaves) * 25, seed=4)
    its = {}
    for st in (True, False):
        H = AdaptiveHierarchy(2, 8, 2, leaves, 4, HierarchyOptions(spacetree_levels=st))
        u, hist = H.solve(b, rtol=1e-10, maxit=300)
        assert hist[-1] <= 1e-10 * hist[0]
        its[st] = len(hist) - 1
    assert its[True] <= 30 and its[True] < its[False] / 2, its
