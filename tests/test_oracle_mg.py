"""Pins of the oracle's multigrid components (paper Section 5) against
Galerkin identities, independent assembly and brute-force solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import SIPG, Hierarchy, HierarchyOptions, q1_stiffness, manufactured as mf
from oracle.mg import (cg_prolongation, cg_to_dg_prolongation, coarse_vertex_positions, extract_diagonal_blocks,
                       dg_to_dg_prolongation, hat_prolongation_1d, p_levels)


def test_p_schedule():
    assert p_levels(4) == [4, 2]
    assert p_levels(5) == [5, 2]
    assert p_levels(3) == [3]
    assert p_levels(8) == [8, 4, 2]
    assert p_levels(1) == [1]


@pytest.mark.parametrize("n", [4, 5, 7, 8, 9])
def test_hat_prolongation_reproduces_linears(n):
    P = hat_prolongation_1d(n)
    pos = coarse_vertex_positions(n)
    x_f = np.arange(n + 1) / n
    x_c = pos / n
    assert np.allclose(P @ x_c, x_f)
    assert np.allclose(P @ np.ones(len(pos)), 1.0)
    assert pos[0] == 0 and pos[-1] == n


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (2, 3, 3), (3, 3, 1), (3, 2, 3)])
def test_dg_to_cg_galerkin_is_q1_stiffness(dim, n, p):
    # P^T A_DG P = Q1 stiffness: face terms vanish on continuous functions
    # with zero boundary values (paper Section 2.4).
    kappa = synth.kappa_log_uniform(dim, n, seed=21)
    s = SIPG(dim, n, p, kappa)
    P = cg_to_dg_prolongation(s)
    G = (P.T @ s.A @ P).toarray()
    Q = q1_stiffness(dim, n, kappa).toarray()
    assert np.abs(G - Q).max() < 1e-11 * np.abs(Q).max()


@pytest.mark.parametrize("dim,n,p,q", [(2, 3, 4, 2), (3, 2, 4, 2), (2, 3, 3, 1)])
def test_dg_to_dg_galerkin_equals_rediscretisation(dim, n, p, q):
    # nested spaces + the same bilinear form (fine-level penalty) => equal
    kappa = synth.kappa_log_uniform(dim, n, seed=22)
    s = SIPG(dim, n, p, kappa)
    P = dg_to_dg_prolongation(s, q)
    G = (P.T @ s.A @ P).toarray()
    R = SIPG(dim, n, q, kappa, p_penalty=p).A.toarray()
    assert np.abs(G - R).max() < 1e-11 * np.abs(R).max()


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 3, 3)])
def test_cg_to_dg_interpolates_trilinears(dim, n, p):
    s = SIPG(dim, n, p)
    P = cg_to_dg_prolongation(s)
    nv = n - 1
    idx = np.arange(nv ** dim)
    V = np.stack([((idx // nv ** k) % nv + 1) / n for k in range(dim)], axis=1)

    # arbitrary vertex values; P must reproduce their Q1 interpolant at DG nodes
    gv = np.prod(np.minimum(V, 1 - V), axis=1) + V[:, 0] ** 2
    u = P @ gv
    # check against direct trilinear interpolation inside each cell
    X = s.dof_coords()
    cell = np.minimum((X * n).astype(int), n - 1)
    t = X * n - cell
    val = np.zeros(len(X))
    for corner in range(2 ** dim):
        bits = np.array([(corner >> k) & 1 for k in range(dim)])
        w = np.prod(np.where(bits, t, 1 - t), axis=1)
        vv = cell + bits
        inside = np.all((vv > 0) & (vv < n), axis=1)
        vid = np.sum((vv - 1) * (nv ** np.arange(dim)), axis=1)
        val += np.where(inside, w * gv[np.where(inside, vid, 0)], 0.0)
    assert np.abs(u - val).max() < 1e-13


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 6), (3, 5)])
def test_cg_galerkin_coarse_operator(dim, n):
    # Coarse Q1 operator by P^T A P equals Q1 rediscretisation for even n
    A = q1_stiffness(dim, n)
    P = cg_prolongation(dim, n)
    G = (P.T @ A @ P).toarray()
    if n % 2 == 0:
        Q = q1_stiffness(dim, n // 2).toarray()
        assert np.abs(G - Q).max() < 1e-12 * np.abs(Q).max()
    # always symmetric positive definite
    assert np.abs(G - G.T).max() < 1e-13 * np.abs(G).max()
    np.linalg.cholesky(G)


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 3, 2)])
def test_block_jacobi_contracts(dim, n, p):
    # rho(I - omega D^-1 A) < 1 for the block-Jacobi smoother (omega = 0.7)
    H = Hierarchy(dim, n, p, synth.kappa_log_uniform(dim, n, seed=4))
    lev = H.levels[0]
    A = lev.A.toarray()
    Dinv = np.zeros_like(A)
    nd = lev.nd
    for c in range(A.shape[0] // nd):
        sl = slice(c * nd, (c + 1) * nd)
        Dinv[sl, sl] = np.linalg.inv(A[sl, sl])
    E = np.eye(A.shape[0]) - H.opts.omega_dg * Dinv @ A
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0


@pytest.mark.parametrize("dim,n,p,var", [(2, 8, 2, False), (2, 6, 3, True), (3, 4, 2, False), (3, 3, 3, True)])
def test_mg_pcg_equals_direct_solve(dim, n, p, var):
    kappa = synth.kappa_log_uniform(dim, n, seed=9) if var else None
    H = Hierarchy(dim, n, p, kappa)
    b = synth.random_rhs(H.fine.ndof, seed=10)
    x, hist = H.solve(b, rtol=1e-12, maxit=300)
    xd = spla.spsolve(H.fine.A.tocsc(), b)
    assert hist[-1] <= 1e-12 * hist[0]
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()


def test_vcycle_on_coarsest_is_exact():
    H = Hierarchy(2, 4, 1)
    last = len(H.levels) - 1
    A = H.levels[last].A.toarray()
    b = synth.random_rhs(A.shape[0], seed=1)
    x = H.vcycle(last, np.zeros_like(b), b)
    assert np.allclose(A @ x, b, atol=1e-12)


def test_vcycle_is_h_robust_2d():
    # the V-cycle contraction does not degrade with h (paper Section 6.3)
    rates = []
    for n in [8, 16, 32]:
        H = Hierarchy(2, n, 2)
        u, f = mf.sin_product(2, 1)
        b = H.fine.load_vector(f)
        _, hist, _ = H.mgmult(b, rtol=1e-7, maxit=100)
        rates.append(len(hist) - 1)
    assert max(rates) - min(rates) <= 3, rates
    assert max(rates) < 40, rates


def test_p_schedule_direct():
    # one-step p-coarsening DG_p -> Q1 (the paper's two-grid hp scheme)
    for p in range(1, 9):
        assert p_levels(p, mode="direct") == [p]


@pytest.mark.parametrize("n", [3, 9, 10, 11, 27])
def test_hat_prolongation_factor3_reproduces_linears(n):
    P = hat_prolongation_1d(n, 3)
    pos = coarse_vertex_positions(n, 3)
    assert pos[0] == 0 and pos[-1] == n
    assert np.all(np.diff(pos) <= 3) and np.all(np.diff(pos) >= 1)
    assert np.allclose(P @ (pos / n), np.arange(n + 1) / n)
    assert np.allclose(P.sum(axis=1), 1.0)
    # a fine vertex between two coarse ones takes weights 1/3, 2/3
    if n % 3 == 0:
        assert np.allclose(P[1, :2], [2 / 3, 1 / 3])


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 6), (2, 10)])
def test_cg_galerkin_factor3(dim, n):
    # P^T A P with factor-3 transfers equals the Q1 stiffness on n/3 cells
    # (independent Q1 assembly) when 3 divides n; SPD always
    A = q1_stiffness(dim, n)
    P = cg_prolongation(dim, n, 3)
    G = (P.T @ A @ P).toarray()
    if n % 3 == 0:
        Q = q1_stiffness(dim, n // 3).toarray()
        assert np.abs(G - Q).max() < 1e-12 * np.abs(Q).max()
    assert np.abs(G - G.T).max() < 1e-13 * np.abs(G).max()
    np.linalg.cholesky(G)


def test_direct_hierarchy_levels():
    H = Hierarchy(2, 9, 4, opts=HierarchyOptions(p_coarsening="direct", h_factor=3, coarsest_n=3))
    kinds = [(lev.kind, lev.n) for lev in H.levels]
    assert kinds == [("dg", 9), ("cg", 9), ("cg", 3)]


def test_mgmult_histories_match_iteration_matrix():
    # MGMult is the linear stationary iteration u_k = u_{k-1} + M (b - A u_{k-1})
    # with M the V-cycle from zero: build M column by column and check both
    # residual histories and the two exit criteria against matrix powers
    opts = HierarchyOptions(p_coarsening="direct", h_factor=3, coarsest_n=3, nu_post=0)
    H = Hierarchy(2, 3, 2, opts=opts)
    A = H.levels[0].A.toarray()
    nd = A.shape[0]
    M = np.stack([H.vcycle(0, np.zeros(nd), e) for e in np.eye(nd)], axis=1)
    b = synth.random_rhs(nd, seed=71)
    u = np.zeros(nd)
    hist, phist = [np.linalg.norm(b)], []
    for _ in range(12):
        du = M @ (b - A @ u)
        u = u + du
        phist.append(np.linalg.norm(du))
        hist.append(np.linalg.norm(b - A @ u))
    _, h2, p2 = H.mgmult(b, rtol=1e-30, maxit=12)
    assert np.allclose(h2, hist, rtol=1e-9, atol=0)
    assert np.allclose(p2, phist, rtol=1e-9, atol=0)
    tol = phist[5] / phist[0] * 1.0000001
    _, _, p3 = H.mgmult(b, rtol=tol, maxit=50, exit="prec")
    assert len(p3) == 6
    tolu = hist[4] / hist[0] * 1.0000001
    _, h4, _ = H.mgmult(b, rtol=tolu, maxit=50, exit="unprec")
    assert len(h4) == 5


def test_paper_mode_is_h_robust_2d():
    # one-step p-coarsening, factor-3 h-coarsening, MGMult: cycle counts to
    # 1e-7 settle as h shrinks (unpreconditioned exit) and do not grow
    # (preconditioned exit), the paper's robustness result (Section 6)
    unprec, prec = [], []
    for n in [9, 27, 81]:
        opts = HierarchyOptions(p_coarsening="direct", h_factor=3, coarsest_n=3)
        H = Hierarchy(2, n, 2, opts=opts)
        _, f = mf.sin_product(2, 2)
        b = H.fine.load_vector(f)
        _, hist, _ = H.mgmult(b, rtol=1e-7, maxit=100)
        _, _, ph = H.mgmult(b, rtol=1e-7, maxit=100, exit="prec")
        unprec.append(len(hist) - 1)
        prec.append(len(ph))
    assert abs(unprec[2] - unprec[1]) <= 1, unprec
    assert prec[0] >= prec[1] >= prec[2], prec


def test_gauss_legendre_hierarchy_solves():
    # MG-PCG with Gauss-Legendre nodes on every DG level reaches the direct
    # solution; the V-cycle contracts as with Gauss-Lobatto nodes
    for basis in ("gll", "gl"):
        H = Hierarchy(2, 6, 4, synth.kappa_log_uniform(2, 6, seed=9), opts=HierarchyOptions(basis=basis))
        b = synth.random_rhs(H.fine.ndof, seed=10)
        u, hist = H.solve(b, rtol=1e-10, maxit=100)
        ref = spla.spsolve(H.levels[0].A.tocsc(), b)
        assert np.abs(u - ref).max() <= 1e-8 * np.abs(ref).max()
        assert len(hist) - 1 < 40


@pytest.mark.parametrize("dim,n,p", [(2, 4, 3), (3, 3, 2)])
def test_interior_block_variant(dim, n, p):
    # every interior cell has the same block for constant kappa; the
    # interior-block smoother differs from the exact one only on boundary
    # cells, still contracts, and MGMult with it reaches the direct solution
    H = Hierarchy(dim, n, p, 1.7)
    blocks = extract_diagonal_blocks(H.levels[0].A, (p + 1) ** dim)
    cc = H.fine.cell_index_coords()
    interior = np.all((cc > 0) & (cc < n - 1), axis=1)
    ref = blocks[np.nonzero(interior)[0][0]]
    assert all(np.abs(blocks[c] - ref).max() <= 1e-13 * np.abs(ref).max() for c in np.nonzero(interior)[0])
    Hi = Hierarchy(dim, n, p, 1.7, opts=HierarchyOptions(block="interior"))
    A = Hi.levels[0].A.toarray()
    nd = A.shape[0]
    D = np.zeros_like(A)
    bs = (p + 1) ** dim
    for c in range(nd // bs):
        D[c * bs:(c + 1) * bs, c * bs:(c + 1) * bs] = ref
    E = np.eye(nd) - 0.7 * np.linalg.solve(D, A)
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0
    b = synth.random_rhs(nd, seed=81)
    u, hist, _ = Hi.mgmult(b, rtol=1e-10, maxit=300)
    assert hist[-1] <= 1e-10 * hist[0]
    assert np.abs(A @ u - b).max() <= 1e-8 * np.abs(b).max()
