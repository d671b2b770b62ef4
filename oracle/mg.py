"""Multigrid oracle on assembled matrices (test infrastructure only).

Written from the paper's Section 5 (Algorithms CoarseGridCorrection and
MGMult; the h-multigrid V-cycle of Section 5.2) and Section 2.3.2
(block-Jacobi, eq. block-Jacobi-IP) / Section 2.4 (point-Jacobi on CG_1),
with these readings where the paper is silent or ambiguous:

* p-coarsening halves p (floor) while the halved degree is >= 2, then goes
  to the continuous Q1 space (zero boundary values) on the same mesh;
* h-coarsening of Q1 by a factor of two (option: three, the paper's factor
  for its 3^k meshes); a cell count that is not a multiple keeps the last
  fine vertex as a coarse vertex, so the coarse spaces stay nested;
  coarsening stops once n <= coarsest_n (4);
* option: p-coarsening straight from DG_p to Q1 in one step (the paper's
  two-grid hp scheme) instead of halving p;
* every transfer is nodal interpolation P (coarse function evaluated at the
  fine nodes) and restriction is P^T; every coarse operator is the Galerkin
  product P^T A P;
* V(nu1, nu2) cycle, block-Jacobi with the exact diagonal blocks A_{K<-K}
  (dense Cholesky) on DG levels, point-Jacobi with diag(A) on Q1 levels,
  dense Cholesky on the coarsest level; the DG and the Q1 levels have their
  own smoothing counts, so that the DG level can run Algorithm MGMult's nu
  pre- and zero post-smoothing steps while the Q1 h-multigrid of Section 5.2
  pre- and post-smooths;
* solve: multigrid-preconditioned (flexible) CG in FP64 to a relative
  unpreconditioned residual ||b - A u|| <= rtol ||b - A u0||.

Pinned by tests/test_oracle_mg.py: Galerkin identities, exactness of the
coarse solve on tiny meshes, dense direct solve equal to the MG-PCG result,
contraction of the smoother iteration matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import lagrange_1d
from .sipg import SIPG, _kron_dims


@dataclass
class HierarchyOptions:
    omega_dg: float = 0.7
    omega_cg: float = 2.0 / 3.0
    nu_pre: int = 2              # block-Jacobi steps before / after the coarse correction on DG levels
    nu_post: int = 2             # (Algorithm MGMult: nu_pre = nu, nu_post = 0)
    nu_pre_cg: int | None = None   # point-Jacobi steps on Q1 levels (Section 5.2: pre-smoothing, then a
    nu_post_cg: int | None = None  # few post-smoothing steps); None: the DG counts
    sigma0: float = 2.0
    coarsest_n: int = 4
    p_schedule: list = field(default_factory=list)  # explicit DG degrees after the fine one
    p_coarsening: str = "halve"  # "halve" (gradual) or "direct" (DG_p -> Q1 in one step, Section 5.2)
    h_factor: int = 2            # Q1 h-coarsening factor (2, or 3 as in the paper's meshes 3^k)
    basis: str = "gll"           # DG nodes: "gll" (Gauss-Lobatto) or "gl" (Gauss-Legendre)
    spacetree_levels: bool = True  # adaptive meshes: coarsen the last DG level along the spacetree levels
                                   # (finest leaves merged into their parents, level by level) down to the
                                   # base mesh before Q1; False: straight to Q1 on the base mesh
    block: str = "exact"         # block-Jacobi block: "exact" A_{K<-K}, or "interior": the block of an
                                 # interior cell for every cell (Section 4, technique approximate
                                 # boundary operators; constant kappa, n >= 3)


def p_levels(p: int, schedule=None, mode: str = "halve"):
    """DG degrees of the hierarchy (fine first); Q1 follows the last entry."""
    if schedule:
        return [p] + [q for q in schedule]
    if mode == "direct":
        return [p]
    out = [p]
    q = p // 2
    while q >= 2:
        out.append(q)
        q //= 2
    return out


def coarse_vertex_positions(n: int, factor: int = 2):
    """Fine vertex indices kept as coarse vertices (every factor-th vertex;
    the last vertex is kept when n is not a multiple of factor)."""
    pos = list(range(0, n + 1, factor))
    if pos[-1] != n:
        pos.append(n)
    return np.array(pos)


def hat_prolongation_1d(n: int, factor: int = 2):
    """1D nodal interpolation from the coarse vertex grid to the fine vertices
    0..n (all vertices, boundary included): P[i, I] = hat_I(x_i)."""
    pos = coarse_vertex_positions(n, factor)
    P = np.zeros((n + 1, len(pos)))
    for i in range(n + 1):
        J = np.searchsorted(pos, i)
        if pos[J] == i:
            P[i, J] = 1.0
        else:
            a, b = pos[J - 1], pos[J]
            t = (i - a) / (b - a)
            P[i, J - 1] = 1.0 - t
            P[i, J] = t
    return P


def cg_prolongation(dim: int, n: int, factor: int = 2) -> sp.csr_matrix:
    """Q1 interior vertices of the coarse grid -> interior vertices of n^dim."""
    P1 = hat_prolongation_1d(n, factor)[1:-1, 1:-1]
    return sp.csr_matrix(_kron_dims([P1] * dim))


def dg_to_dg_prolongation(fine: SIPG, q: int) -> sp.csr_matrix:
    """Nodal interpolation Q_q -> Q_p on every cell (same mesh, same node family)."""
    from .basis import gl_nodes, gll_nodes
    coarse_nodes = gll_nodes(q) if fine.basis == "gll" else gl_nodes(q)
    E, _ = lagrange_1d(coarse_nodes, fine.nodes1d)  # E[a, a'] = l^q_{a'}(xi^p_a)
    Pc = _kron_dims([E] * fine.dim)
    return sp.csr_matrix(sp.kron(sp.identity(fine.ncell), sp.csr_matrix(Pc)))


def cg_to_dg_prolongation(fine: SIPG) -> sp.csr_matrix:
    """Q1 (interior vertices) -> DG nodal values: P[(K,i), V] = phi_V(x_{K,i})."""
    d, n, N = fine.dim, fine.n, fine.N
    xi = fine.nodes1d
    nv = n - 1
    cc = fine.cell_index_coords()
    rows, cols, vals = [], [], []
    loc = [(np.arange(fine.nd) // N ** k) % N for k in range(d)]
    for corner in range(2 ** d):
        bits = [(corner >> k) & 1 for k in range(d)]
        w = np.ones(fine.nd)
        for k in range(d):
            w *= xi[loc[k]] if bits[k] else (1.0 - xi[loc[k]])
        v = cc + np.array(bits)[None, :]
        inside = np.all((v > 0) & (v < n), axis=1)
        cells = np.nonzero(inside)[0]
        vid = np.zeros(len(cells), dtype=np.int64)
        for k in range(d):
            vid += (v[cells, k] - 1) * nv ** k
        for i in range(fine.nd):
            if w[i] == 0.0:
                continue
            rows.append(cells * fine.nd + i)
            cols.append(vid)
            vals.append(np.full(len(cells), w[i]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.ndof, nv ** d))


class Level:
    def __init__(self, kind, A, n, p=None, blocks=None):
        self.kind, self.A, self.n, self.p = kind, A.tocsr(), n, p
        self.size = A.shape[0]
        if kind == "dg":
            nd = blocks.shape[1]
            self.nd = nd
            L = np.linalg.cholesky(blocks)
            self.Linv = np.linalg.inv(L)
        else:
            self.diag = self.A.diagonal()

    def block_solve(self, r):
        """D^{-1} r with D = blockdiag(A_{K<-K}) (dense Cholesky factors)."""
        R = r.reshape(-1, self.nd)
        y = np.einsum("cij,cj->ci", self.Linv, R)
        return np.einsum("cji,cj->ci", self.Linv, y).ravel()


def extract_diagonal_blocks(A: sp.spmatrix, nd: int) -> np.ndarray:
    """Diagonal nd x nd blocks of an assembled matrix (block-Jacobi D)."""
    B = sp.bsr_matrix(A, blocksize=(nd, nd))
    nb = A.shape[0] // nd
    out = np.zeros((nb, nd, nd))
    for r in range(nb):
        for k in range(B.indptr[r], B.indptr[r + 1]):
            if B.indices[k] == r:
                out[r] = B.data[k]
    return out


class Hierarchy:
    """hp-multigrid hierarchy DG_p -> DG_{p/2} -> ... -> Q1(n) -> Q1(n/2) ..."""

    def __init__(self, dim, n, p, kappa=None, opts: HierarchyOptions | None = None):
        self.opts = opts or HierarchyOptions()
        self.dim = dim
        fine = SIPG(dim, n, p, kappa, sigma0=self.opts.sigma0, basis=self.opts.basis)
        self.fine = fine
        self.levels = []
        self.P = []  # P[l]: level l+1 -> level l
        A = fine.A.tocsr()
        degs = p_levels(p, self.opts.p_schedule, self.opts.p_coarsening)
        cur = fine
        for li, q in enumerate(degs):
            blocks = extract_diagonal_blocks(A, (q + 1) ** dim)
            if self.opts.block == "interior":
                if n < 3:
                    raise ValueError("the interior-block smoother needs an interior cell (n >= 3)")
                inner = sum(n ** k for k in range(dim))  # cell (1, 1[, 1])
                blocks = np.broadcast_to(blocks[inner], blocks.shape).copy()
            self.levels.append(Level("dg", A, n, q, blocks))
            if li + 1 < len(degs):
                nxt = SIPG(dim, n, degs[li + 1], kappa, p_penalty=p, sigma0=self.opts.sigma0, basis=self.opts.basis)
                P = dg_to_dg_prolongation(cur, degs[li + 1])
                cur = nxt
            else:
                P = cg_to_dg_prolongation(cur)
            self.P.append(P)
            A = (P.T @ A @ P).tocsr()
        m = n
        while True:
            self.levels.append(Level("cg", A, m))
            if m <= self.opts.coarsest_n:
                break
            P = cg_prolongation(dim, m, self.opts.h_factor)
            self.P.append(P)
            A = (P.T @ A @ P).tocsr()
            m = len(coarse_vertex_positions(m, self.opts.h_factor)) - 1
        last = self.levels[-1]
        self.coarse_chol = sla.cho_factor(last.A.toarray())

    # ------------------------------------------------------------- smoothers
    def smoothing_counts(self, l):
        """(pre, post) smoothing steps on level l."""
        o = self.opts
        if self.levels[l].kind == "dg":
            return o.nu_pre, o.nu_post
        return (o.nu_pre if o.nu_pre_cg is None else o.nu_pre_cg,
                o.nu_post if o.nu_post_cg is None else o.nu_post_cg)

    def smooth(self, l, u, b, nsweeps):
        lev = self.levels[l]
        for _ in range(nsweeps):
            r = b - lev.A @ u
            if lev.kind == "dg":
                u = u + self.opts.omega_dg * lev.block_solve(r)
            else:
                u = u + self.opts.omega_cg * r / lev.diag
        return u

    def vcycle(self, l, u, b):
        """One V-cycle on level l starting from u: pre-smoothing, coarse
        correction (one V-cycle on the next level from zero), post-smoothing."""
        if l == len(self.levels) - 1:
            return sla.cho_solve(self.coarse_chol, b)
        pre, post = self.smoothing_counts(l)
        u = self.smooth(l, u, b, pre)
        r = b - self.levels[l].A @ u
        P = self.P[l]
        e = self.vcycle(l + 1, np.zeros(P.shape[1]), P.T @ r)
        u = u + P @ e
        return self.smooth(l, u, b, post)

    def precondition(self, r):
        return self.vcycle(0, np.zeros_like(r), r)

    # ---------------------------------------------------------------- solver
    def solve(self, b, rtol=1e-10, maxit=200, u0=None, flexible=True):
        """MG-preconditioned CG; returns (u, residual history)."""
        A = self.levels[0].A
        u = np.zeros_like(b) if u0 is None else u0.copy()
        r = b - A @ u
        r0 = np.linalg.norm(r)
        hist = [r0]
        if r0 == 0.0:
            return u, hist
        z = self.precondition(r)
        pdir = z.copy()
        rz = r @ z
        for _ in range(maxit):
            q = A @ pdir
            alpha = rz / (pdir @ q)
            u += alpha * pdir
            r_new = r - alpha * q
            hist.append(np.linalg.norm(r_new))
            if hist[-1] <= rtol * r0:
                break
            z_new = self.precondition(r_new)
            if flexible:
                beta = (z_new @ (r_new - r)) / rz
            else:
                beta = (z_new @ r_new) / rz
            rz = z_new @ r_new
            pdir = z_new + beta * pdir
            r, z = r_new, z_new
        return u, hist

    def mgmult(self, b, rtol=1e-10, maxit=200, u0=None, exit="unprec"):
        """Stationary multigrid iteration u <- V(u, b) (Algorithm MGMult with a
        V(nu1, nu2) cycle); returns (u, unpreconditioned residual history,
        preconditioned residual history ||u_k - u_{k-1}||).  Exit (Section
        5.1.1): "unprec" once ||b - A u_k|| <= rtol ||b - A u_0||, "prec" once
        the preconditioned residual ||u_k - u_{k-1}|| <= rtol ||u_1 - u_0||."""
        A = self.levels[0].A
        u = np.zeros_like(b) if u0 is None else u0.copy()
        r0 = np.linalg.norm(b - A @ u)
        hist, phist = [r0], []
        for _ in range(maxit):
            un = self.vcycle(0, u, b)
            phist.append(np.linalg.norm(un - u))
            u = un
            hist.append(np.linalg.norm(b - A @ u))
            if exit == "prec":
                if phist[-1] <= rtol * phist[0]:
                    break
            elif hist[-1] <= rtol * r0:
                break
        return u, hist, phist
