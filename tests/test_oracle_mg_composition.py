"""Pins of the composition of the oracle's V-cycle and of Algorithm MGMult
(paper Section 5: Algorithm CoarseGridCorrection, Algorithm MGMult and the
hp-multigrid of Section 5.2).

The expected operators are built densely from the fine matrix A_0 and the
transfers P_l alone (both pinned elsewhere), by the textbook recursion for
the error propagation of a V-cycle with an exact coarsest solve:

    E_L = 0,
    E_l = S_l^post (I - P_l (I - E_{l+1}) A_{l+1}^{-1} P_l^T A_l) S_l^pre,
    A_{l+1} = P_l^T A_l P_l,  S_l = I - omega_l D_l^{-1} A_l,

with D_l the cell blocks (DG levels) or the diagonal (Q1 levels) sliced out
of the dense A_l.  The oracle's recursive code is read only through its
action on unit vectors: E[:, j] = V(e_j, 0) and B[:, j] = V(0, e_j).
Mutation checks plant the plausible mistakes (V(2,0) for V(2,2), the DG and
Q1 relaxation factors or smoothing counts exchanged) in the oracle and
confirm that the identities see them.
"""
import numpy as np
import pytest

import synth
from oracle import Hierarchy, HierarchyOptions


def _dense(M):
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M)


def smoother(A, kind, bs, omega):
    """I - omega D^{-1} A with D sliced out of the dense A."""
    n = A.shape[0]
    Dinv = np.zeros_like(A)
    if kind == "dg":
        for c in range(n // bs):
            sl = slice(c * bs, (c + 1) * bs)
            Dinv[sl, sl] = np.linalg.inv(A[sl, sl])
    else:
        Dinv[np.diag_indices(n)] = 1.0 / np.diag(A)
    return np.eye(n) - omega * Dinv @ A


def textbook_E(A0, Ps, kinds, bss, counts, omegas):
    """Error propagation of the V-cycle on level 0 (see module docstring)."""
    As = [A0]
    for P in Ps:
        As.append(P.T @ As[-1] @ P)
    L = len(As) - 1
    E = np.zeros_like(As[L])
    for l in range(L - 1, -1, -1):
        A, P = As[l], Ps[l]
        S = smoother(A, kinds[l], bss[l], omegas[l])
        pre, post = counts[l]
        Binv_c = (np.eye(As[l + 1].shape[0]) - E) @ np.linalg.inv(As[l + 1])
        C = np.eye(A.shape[0]) - P @ Binv_c @ P.T @ A
        E = np.linalg.matrix_power(S, post) @ C @ np.linalg.matrix_power(S, pre)
    return E


def expected_for(H, opts):
    """Textbook E for the level structure of H, with counts and omegas taken
    from `opts` (not from H)."""
    A0 = _dense(H.fine.A)
    Ps = [_dense(P) for P in H.P]
    kinds = [lev.kind for lev in H.levels[:-1]]
    bss = [((lev.p + 1) ** H.dim if lev.kind == "dg" else 1) for lev in H.levels[:-1]]
    cg_pre = opts.nu_pre if opts.nu_pre_cg is None else opts.nu_pre_cg
    cg_post = opts.nu_post if opts.nu_post_cg is None else opts.nu_post_cg
    counts = [(opts.nu_pre, opts.nu_post) if k == "dg" else (cg_pre, cg_post) for k in kinds]
    omegas = [opts.omega_dg if k == "dg" else opts.omega_cg for k in kinds]
    return textbook_E(A0, Ps, kinds, bss, counts, omegas)


def oracle_E(H):
    nd = H.fine.ndof
    z = np.zeros(nd)
    return np.stack([H.vcycle(0, e, z) for e in np.eye(nd)], axis=1)


def oracle_B(H):
    nd = H.fine.ndof
    z = np.zeros(nd)
    return np.stack([H.vcycle(0, z, e) for e in np.eye(nd)], axis=1)


def rel(X, Y):
    return np.abs(X - Y).max() / max(np.abs(Y).max(), 1e-300)


# (dim, n, p, kappa seed or None, options): two-level DG_1 -> Q1; three DG
# levels; DG -> Q1 -> Q1 with Q1 smoothing; variable kappa; paper mode
CASES = [
    (2, 4, 1, None, dict(nu_pre=2, nu_post=2)),
    (2, 4, 1, None, dict(nu_pre=3, nu_post=1, omega_dg=0.8)),
    (2, 4, 4, None, dict(nu_pre=2, nu_post=1, omega_dg=0.75)),
    (2, 8, 2, None, dict(nu_pre=2, nu_post=1, nu_pre_cg=1, nu_post_cg=3, omega_dg=0.8, omega_cg=0.6)),
    (2, 6, 3, 31, dict(nu_pre=1, nu_post=2, nu_pre_cg=2, nu_post_cg=1, omega_dg=0.7, omega_cg=0.55)),
    (2, 9, 2, None, dict(nu_pre=2, nu_post=0, nu_pre_cg=1, nu_post_cg=1, p_coarsening="direct", h_factor=3,
                         coarsest_n=3)),
    (3, 3, 2, 32, dict(nu_pre=2, nu_post=2)),
]


def _hier(dim, n, p, seed, kw):
    kappa = synth.kappa_log_uniform(dim, n, seed=seed) if seed is not None else None
    opts = HierarchyOptions(**kw)
    return Hierarchy(dim, n, p, kappa, opts=opts), opts


@pytest.mark.parametrize("dim,n,p,seed,kw", CASES)
def test_vcycle_error_propagation_is_textbook(dim, n, p, seed, kw):
    H, opts = _hier(dim, n, p, seed, kw)
    assert len(H.levels) >= 2
    E = oracle_E(H)
    Et = expected_for(H, opts)
    assert rel(E, Et) < 1e-11, rel(E, Et)
    # the cycle is the consistent linear iteration u <- E u + B b with
    # B = (I - E) A^{-1}
    A = _dense(H.fine.A)
    B = oracle_B(H)
    assert rel(B, (np.eye(A.shape[0]) - Et) @ np.linalg.inv(A)) < 1e-9


@pytest.mark.parametrize("dim,n,p,seed,kw", [CASES[2], CASES[3], CASES[4]])
def test_vcycle_composition_mutations_are_seen(dim, n, p, seed, kw):
    # plant the plausible mistakes in the oracle's options and check that the
    # identity above fails for each of them
    H, opts = _hier(dim, n, p, seed, kw)
    Et = expected_for(H, opts)
    mutants = [dict(kw, nu_post=0), dict(kw, nu_pre=kw["nu_pre"] + 1)]
    if "omega_cg" in kw:
        mutants.append(dict(kw, omega_dg=kw["omega_cg"], omega_cg=kw["omega_dg"]))
    if "nu_pre_cg" in kw:
        mutants.append(dict(kw, nu_pre_cg=kw["nu_post_cg"], nu_post_cg=kw["nu_pre_cg"]))
        mutants.append(dict(kw, nu_pre_cg=None, nu_post_cg=None))
    for m in mutants:
        Hm, _ = _hier(dim, n, p, seed, m)
        assert rel(oracle_E(Hm), Et) > 1e-3, m


@pytest.mark.parametrize("dim,n,p,seed,nu", [(2, 4, 4, None, 2), (2, 8, 2, 33, 1), (2, 6, 3, 34, 3),
                                             (3, 3, 2, None, 2)])
def test_symmetric_vcycle_is_spd_preconditioner(dim, n, p, seed, nu):
    # V(nu, nu) with A-self-adjoint Jacobi smoothers gives a symmetric
    # positive definite B; V(nu, 0) does not (control)
    H, _ = _hier(dim, n, p, seed, dict(nu_pre=nu, nu_post=nu))
    B = oracle_B(H)
    assert rel(B, B.T) < 1e-12
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0
    Hn, _ = _hier(dim, n, p, seed, dict(nu_pre=nu, nu_post=0, nu_pre_cg=nu, nu_post_cg=nu))
    Bn = oracle_B(Hn)
    assert rel(Bn, Bn.T) > 1e-3


@pytest.mark.parametrize("dim,n,p,seed,kw", [
    (2, 9, 2, None, dict(nu_pre=2, nu_post=0, nu_pre_cg=1, nu_post_cg=1, p_coarsening="direct", h_factor=3,
                         coarsest_n=3)),
    (2, 8, 3, 35, dict(nu_pre=3, nu_post=0, nu_pre_cg=2, nu_post_cg=2)),
])
def test_mgmult_iterates_are_textbook(dim, n, p, seed, kw):
    # Algorithm MGMult with nu pre- and zero post-smoothing steps: every
    # iterate equals u_k = E u_{k-1} + (I - E) A^{-1} b with the textbook E,
    # and the two residual histories follow
    H, opts = _hier(dim, n, p, seed, kw)
    Et = expected_for(H, opts)
    A = _dense(H.fine.A)
    nd = A.shape[0]
    b = synth.random_rhs(nd, seed=91)
    u0 = synth.random_vector(nd, seed=92)
    xs = np.linalg.solve(A, b)
    u = u0.copy()
    hist, phist = [np.linalg.norm(b - A @ u)], []
    for _ in range(6):
        un = Et @ u + (xs - Et @ xs)
        phist.append(np.linalg.norm(un - u))
        u = un
        hist.append(np.linalg.norm(b - A @ u))
    uo, h2, p2 = H.mgmult(b, rtol=1e-30, maxit=6, u0=u0)
    assert np.abs(uo - u).max() <= 1e-9 * np.abs(u).max()
    assert np.allclose(h2, hist, rtol=1e-8, atol=0)
    assert np.allclose(p2, phist, rtol=1e-8, atol=0)
