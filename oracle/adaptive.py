"""Assembled SIPG operator and hp-multigrid on adaptive (spacetree) meshes
for the oracle (test infrastructure only).

Paper Section 2.1 (hierarchical Cartesian meshes: the leaves of a spacetree
over the unit box form the mesh; every facet is shared by a left and a right
cell, the skeleton is the set of facets between leaves) and Section 2.3
(eq. weak_form_IP) on such meshes.  Readings where the paper is silent:

* spacetree with subdivision factor r (2, or 3 as in the paper) over n^d
  base cells; facet neighbours are at most one level apart (facet balance),
  so a facet is either shared by two leaves of one level (conforming) or is
  the part of a coarse leaf's facet that one finer leaf covers (hanging: a
  coarse facet meets r^(d-1) finer leaves); the skeleton pieces are the
  facets of the finer side;
* the penalty of a piece is sigma = sigma0 (p_pen+1)^2 / min(h-, h+) (the
  finer side's width), 2 sigma0 (p_pen+1)^2 / h_K on boundary facets;
* coarse spaces for the multigrid: the DG spaces of lower degree on the same
  leaves (nodal interpolation, Galerkin products); then, at the last DG
  degree, the DG spaces of the coarser spacetree levels (Section 2.1: coarse
  meshes come from the coarser levels of the spacetree): the leaves of the
  deepest level merged into their parents, one level at a time, down to the
  base mesh, each operator rediscretised on its leaves with the fine
  penalty factor sigma0 (p+1)^2 / h_F and the transfer the nodal
  interpolation of the parent's polynomial; then the continuous Q1 space of
  the base mesh (level 0; vanishing on the boundary), embedded by
  evaluating its trilinear functions at the DG nodes of every leaf, then the
  h-levels of that base mesh as for uniform meshes.

Everything here is the plain definition: every bilinear-form integral is
evaluated in physical coordinates by Gauss quadrature on the facet pieces
and cells, with the basis functions of the two cells evaluated at the same
physical points (no reference-facet tables, no remapping of traces).
Pinned by tests/test_oracle_adaptive.py: a mesh of one level equals the
uniform oracle, symmetry and positive definiteness with hanging facets,
exact reproduction of a polynomial solution (consistency across hanging
facets), annihilation of global linears away from the boundary, Galerkin
product of the base Q1 space equal to the independently assembled Q1
stiffness, MG-PCG equal to a direct solve, manufactured-solution rate p+1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gauss_rule, gl_nodes, gll_nodes, lagrange_1d
from .mg import Hierarchy, HierarchyOptions, Level, cg_prolongation, coarse_vertex_positions, \
    extract_diagonal_blocks, p_levels
from .sipg import _kron_dims


class AdaptiveSIPG:
    """SIPG discretisation of -div(kappa grad u) = f, u = 0 on the boundary,
    on the leaves of a facet-balanced spacetree (leaves: (nleaf, 1 + dim)
    integer rows (level, x_0, ..); cell vectors follow the row order, local
    node index a + N b (+ N^2 c), x fastest)."""

    def __init__(self, dim, n, r, leaves, p, kappa=None, p_penalty=None, sigma0=2.0, basis="gll"):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if r not in (2, 3):
            raise ValueError("subdivision factor must be 2 or 3")
        self.dim, self.n, self.r, self.p = dim, n, r, p
        self.leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 1 + dim)
        self.level = self.leaves[:, 0]
        self.coords = self.leaves[:, 1:]
        self.ncell = len(self.leaves)
        self.N = p + 1
        self.nd = self.N ** dim
        self.ndof = self.ncell * self.nd
        self.h = 1.0 / (n * np.power(float(r), self.level))
        self.origin = self.coords * self.h[:, None]
        if kappa is None:
            kappa = 1.0
        kappa = np.asarray(kappa, dtype=np.float64)
        if kappa.ndim == 0:
            kappa = np.full(self.ncell, float(kappa))
        if kappa.shape != (self.ncell,) or not np.all(kappa > 0):
            raise ValueError("kappa must be positive, one value per leaf")
        self.kappa = kappa
        self.p_penalty = p if p_penalty is None else p_penalty
        self.sigma0 = sigma0
        self.basis = basis
        self.nodes1d = gll_nodes(p) if basis == "gll" else gl_nodes(p)
        self.index = {(int(l),) + tuple(int(v) for v in x): i for i, (l, x) in
                      enumerate(zip(self.level, self.coords))}
        if len(self.index) != self.ncell:
            raise ValueError("duplicate leaves")
        vol = np.sum(self.h ** dim)
        if abs(vol - 1.0) > 1e-12:
            raise ValueError("the leaves do not tile the unit box")
        self._A = None
        self.pieces = self._facet_pieces()

    # ------------------------------------------------------------ geometry
    def _leaf(self, lvl, x):
        return self.index.get((lvl,) + tuple(x))

    def _facet_pieces(self):
        """Skeleton pieces (minus cell, plus cell or -1, axis k, boundary side
        (+1 / -1, 0 if interior), width hF of the piece, lower corner of the
        piece).  Interior pieces are found from the + facet of every leaf."""
        d, n, r = self.dim, self.n, self.r
        out = []
        for K in range(self.ncell):
            lvl, x, h = int(self.level[K]), self.coords[K], self.h[K]
            ext = n * r ** lvl
            for k in range(d):
                if x[k] == 0:
                    out.append((K, -1, k, -1, h, self.origin[K].copy()))
                y = x.copy()
                y[k] += 1
                corner = self.origin[K].copy()
                corner[k] += h
                if y[k] == ext:
                    out.append((K, -1, k, +1, h, corner))
                    continue
                nb = self._leaf(lvl, y)
                if nb is not None:
                    out.append((K, nb, k, 0, h, corner))
                    continue
                if lvl > 0:
                    nb = self._leaf(lvl - 1, y // r)
                    if nb is not None:
                        out.append((K, nb, k, 0, h, corner))
                        continue
                # the neighbour region is refined: its children on the facet
                tang = [t for t in range(d) if t != k]
                for m in range(r ** (d - 1)):
                    z = r * y
                    for j, t in enumerate(tang):
                        z[t] += (m // r ** j) % r
                    ch = self._leaf(lvl + 1, z)
                    if ch is None:
                        raise ValueError("facet neighbours more than one level apart")
                    cc = corner.copy()
                    for t in tang:
                        cc[t] = z[t] * self.h[ch]
                    out.append((K, ch, k, 0, self.h[ch], cc))
        return out

    def dof_coords(self):
        """Physical coordinates of every nodal degree of freedom (ndof, dim)."""
        xi = self.nodes1d
        loc = np.stack([xi[(np.arange(self.nd) // self.N ** k) % self.N] for k in range(self.dim)], axis=1)
        X = self.origin[:, None, :] + loc[None, :, :] * self.h[:, None, None]
        return X.reshape(-1, self.dim)

    def eval_basis(self, K, X):
        """Values V[q, i] and gradients G[q, i, k] of the basis of leaf K at
        the physical points X (q, dim)."""
        d, N = self.dim, self.N
        xi = (X - self.origin[K][None, :]) / self.h[K]
        V1, D1 = [], []
        for k in range(d):
            v, dv = lagrange_1d(self.nodes1d, xi[:, k])
            V1.append(v)
            D1.append(dv / self.h[K])
        idx = [(np.arange(self.nd) // N ** k) % N for k in range(d)]
        V = np.ones((X.shape[0], self.nd))
        for k in range(d):
            V *= V1[k][:, idx[k]]
        G = np.ones((X.shape[0], self.nd, d))
        for g in range(d):
            for k in range(d):
                G[:, :, g] *= (D1[k] if k == g else V1[k])[:, idx[k]]
        return V, G

    # ------------------------------------------------------------- assembly
    @property
    def A(self) -> sp.csr_matrix:
        if self._A is None:
            self._A = self._assemble()
        return self._A

    def _volume_block(self, K):
        """kappa_K int grad phi_j . grad phi_i over leaf K, Gauss (p+1)^d."""
        d, N = self.dim, self.N
        xq, wq = gauss_rule(N)
        Q = np.stack([xq[(np.arange(N ** d) // N ** k) % N] for k in range(d)], axis=1)
        Wq = np.ones(N ** d)
        for k in range(d):
            Wq *= wq[(np.arange(N ** d) // N ** k) % N]
        X = self.origin[K][None, :] + Q * self.h[K]
        _, G = self.eval_basis(K, X)
        w = Wq * self.h[K] ** d
        return self.kappa[K] * sum((G[:, :, k] * w[:, None]).T @ G[:, :, k] for k in range(d))

    def _piece_blocks(self, piece):
        """Blocks of one skeleton piece: [(row cell, column cell, block)]."""
        d, N = self.dim, self.N
        Km, Kp, k, side, hF, corner = piece
        xq1, wq1 = gauss_rule(N)
        Qf = np.stack([xq1[(np.arange(N ** (d - 1)) // N ** j) % N] for j in range(d - 1)], axis=1)
        Wf = np.ones(N ** (d - 1))
        for j in range(d - 1):
            Wf *= wq1[(np.arange(N ** (d - 1)) // N ** j) % N]
        pen = self.sigma0 * (self.p_penalty + 1) ** 2
        tang = [t for t in range(d) if t != k]
        X = np.repeat(corner[None, :], len(Wf), axis=0)
        for j, t in enumerate(tang):
            X[:, t] += Qf[:, j] * hF
        w = Wf * hF ** (d - 1)
        Vm, Gm = self.eval_basis(Km, X)
        if side != 0:
            # boundary facet: outward normal side * e_k
            Dn = side * Gm[:, :, k]
            sig = 2.0 * pen / self.h[Km]
            WV = Vm * w[:, None]
            return [(Km, Km, self.kappa[Km] * (-WV.T @ Dn - (Dn * w[:, None]).T @ Vm + sig * WV.T @ Vm))]
        Vp, Gp = self.eval_basis(Kp, X)
        Dm, Dp = Gm[:, :, k], Gp[:, :, k]  # derivative along n_F = +e_k
        kF = 2.0 * self.kappa[Km] * self.kappa[Kp] / (self.kappa[Km] + self.kappa[Kp])
        sig = pen / min(self.h[Km], self.h[Kp])

        def m(a, b):  # int a_i b_j over the piece
            return (a * w[:, None]).T @ b

        # a(phi_j, phi_i) with [v] = v- - v+, {dn v} = (dn v- + dn v+)/2
        return [(Km, Km, kF * (-0.5 * m(Vm, Dm) - 0.5 * m(Dm, Vm) + sig * m(Vm, Vm))),
                (Km, Kp, kF * (-0.5 * m(Vm, Dp) + 0.5 * m(Dm, Vp) - sig * m(Vm, Vp))),
                (Kp, Km, kF * (0.5 * m(Vp, Dm) - 0.5 * m(Dp, Vm) - sig * m(Vp, Vm))),
                (Kp, Kp, kF * (0.5 * m(Vp, Dp) + 0.5 * m(Dp, Vp) + sig * m(Vp, Vp)))]

    def _assemble(self):
        nd = self.nd
        rows, cols, vals = [], [], []

        def add(I, J, B):
            ii, jj = np.meshgrid(np.arange(nd) + I * nd, np.arange(nd) + J * nd, indexing="ij")
            rows.append(ii.ravel())
            cols.append(jj.ravel())
            vals.append(B.ravel())

        for K in range(self.ncell):
            add(K, K, self._volume_block(K))
        for piece in self.pieces:
            for I, J, B in self._piece_blocks(piece):
                add(I, J, B)
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.ndof, self.ndof))

    def row_blocks(self, cells):
        """The rows of A belonging to the given leaves, assembled from the
        same volume and piece blocks without the rest of the matrix: a dict
        cell -> {column cell: block} (for sampled checks on large meshes)."""
        want = set(int(c) for c in cells)
        out = {c: {c: self._volume_block(c)} for c in want}
        for piece in self.pieces:
            if piece[0] not in want and piece[1] not in want:
                continue
            for I, J, B in self._piece_blocks(piece):
                if I in want:
                    out[I][J] = out[I].get(J, 0.0) + B
        return out

    def load_vector(self, f, nq=None):
        """b_i = int f phi_i, (p+3)-point Gauss per direction on every leaf."""
        d = self.dim
        nq = self.N + 2 if nq is None else nq
        xq, wq = gauss_rule(nq)
        Q = np.stack([xq[(np.arange(nq ** d) // nq ** k) % nq] for k in range(d)], axis=1)
        Wq = np.ones(nq ** d)
        for k in range(d):
            Wq *= wq[(np.arange(nq ** d) // nq ** k) % nq]
        b = np.zeros(self.ndof)
        for K in range(self.ncell):
            X = self.origin[K][None, :] + Q * self.h[K]
            V, _ = self.eval_basis(K, X)
            b[K * self.nd:(K + 1) * self.nd] = V.T @ (Wq * self.h[K] ** d * f(X))
        return b

    def interpolate(self, u):
        """Nodal interpolant of the function u(X) (X: (m, dim))."""
        return u(self.dof_coords())

    def l2_error(self, uh, u, nq=None):
        """||u_h - u||_L2 by (p+3)-point Gauss per direction on every leaf."""
        d = self.dim
        nq = self.N + 2 if nq is None else nq
        xq, wq = gauss_rule(nq)
        Q = np.stack([xq[(np.arange(nq ** d) // nq ** k) % nq] for k in range(d)], axis=1)
        Wq = np.ones(nq ** d)
        for k in range(d):
            Wq *= wq[(np.arange(nq ** d) // nq ** k) % nq]
        err = 0.0
        for K in range(self.ncell):
            X = self.origin[K][None, :] + Q * self.h[K]
            V, _ = self.eval_basis(K, X)
            e = V @ uh[K * self.nd:(K + 1) * self.nd] - u(X)
            err += np.sum(Wq * self.h[K] ** d * e * e)
        return float(np.sqrt(err))

    # ------------------------------------------------------------ transfers
    def dg_prolongation(self, q):
        """Nodal interpolation Q_q -> Q_p on every leaf."""
        coarse = gll_nodes(q) if self.basis == "gll" else gl_nodes(q)
        E, _ = lagrange_1d(coarse, self.nodes1d)
        Pc = _kron_dims([E] * self.dim)
        return sp.csr_matrix(sp.kron(sp.identity(self.ncell), sp.csr_matrix(Pc)))

    def base_q1_prolongation(self):
        """Continuous Q1 on the base mesh (interior vertices, x fastest) ->
        DG nodal values: P[(K, i), v] = hat_v(x_{K,i})."""
        d, n = self.dim, self.n
        X = self.dof_coords() * n  # base-mesh units
        B = np.minimum(np.floor(X).astype(np.int64), n - 1)
        T = X - B
        nv = n - 1
        rows, cols, vals = [], [], []
        for corner in range(2 ** d):
            bits = [(corner >> k) & 1 for k in range(d)]
            w = np.ones(len(X))
            vid = np.zeros(len(X), dtype=np.int64)
            inside = np.ones(len(X), dtype=bool)
            for k in range(d):
                w *= T[:, k] if bits[k] else 1.0 - T[:, k]
                v = B[:, k] + bits[k]
                inside &= (v > 0) & (v < n)
                vid += (v - 1) * nv ** k
            keep = inside & (w != 0.0)
            rows.append(np.nonzero(keep)[0])
            cols.append(vid[keep])
            vals.append(w[keep])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.ndof, nv ** d))


def coarser_leaves(leaves, r):
    """One spacetree level up: every leaf of the deepest level replaced by
    its parent (each parent listed once, where its first child was); the
    other leaves unchanged.  Returns (coarse leaves, parent index of every
    fine leaf)."""
    leaves = np.asarray(leaves, dtype=np.int64)
    lmax = int(leaves[:, 0].max())
    out, where, parent = [], {}, np.empty(len(leaves), dtype=np.int64)
    for i, row in enumerate(leaves):
        key = tuple(int(v) for v in row)
        if key[0] == lmax and lmax > 0:
            key = (lmax - 1,) + tuple(v // r for v in key[1:])
        if key not in where:
            where[key] = len(out)
            out.append(key)
        parent[i] = where[key]
    return np.array(out, dtype=np.int64), parent


def spacetree_prolongation(fine: AdaptiveSIPG, coarse: AdaptiveSIPG, parent):
    """Nodal interpolation from the coarse leaves to the fine ones: the
    coarse polynomial of the containing leaf evaluated at the fine nodes."""
    X = fine.dof_coords()
    rows, cols, vals = [], [], []
    for K in range(fine.ncell):
        V, _ = coarse.eval_basis(int(parent[K]), X[K * fine.nd:(K + 1) * fine.nd])
        ii, jj = np.nonzero(V != 0.0)
        rows.append(K * fine.nd + ii)
        cols.append(int(parent[K]) * coarse.nd + jj)
        vals.append(V[ii, jj])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.ndof, coarse.ndof))


class AdaptiveHierarchy(Hierarchy):
    """hp-multigrid DG_p -> DG_{p/2} -> ... (on the leaves) -> the last DG
    degree on the coarser spacetree levels (opts.spacetree_levels) -> Q1
    (base mesh) -> Q1 (base mesh / 2) ...; V-cycle, smoothers and solvers of
    Hierarchy."""

    def __init__(self, dim, n, r, leaves, p, opts: HierarchyOptions | None = None, kappa=None):
        self.opts = opts or HierarchyOptions()
        if self.opts.block != "exact":
            raise ValueError("adaptive meshes take the exact cell block")
        self.dim = dim
        fine = AdaptiveSIPG(dim, n, r, leaves, p, kappa, sigma0=self.opts.sigma0, basis=self.opts.basis)
        self.fine = fine
        self.levels, self.P = [], []
        A = fine.A.tocsr()
        degs = p_levels(p, self.opts.p_schedule, self.opts.p_coarsening)
        cur = fine
        for li, q in enumerate(degs):
            self.levels.append(Level("dg", A, n, q, extract_diagonal_blocks(A, (q + 1) ** dim)))
            if li + 1 < len(degs):
                P = cur.dg_prolongation(degs[li + 1])
                cur = AdaptiveSIPG(dim, n, r, leaves, degs[li + 1], kappa, p_penalty=p, sigma0=self.opts.sigma0,
                                   basis=self.opts.basis)
                self.P.append(P)
                A = (P.T @ A @ P).tocsr()
        lv = np.asarray(leaves, dtype=np.int64)
        while self.opts.spacetree_levels and lv[:, 0].max() > 0:
            if kappa is not None and np.ndim(kappa) > 0:
                raise ValueError("spacetree levels take a constant kappa")
            lc, parent = coarser_leaves(lv, r)
            co = AdaptiveSIPG(dim, n, r, lc, cur.p, kappa, p_penalty=p, sigma0=self.opts.sigma0,
                              basis=self.opts.basis)
            self.P.append(spacetree_prolongation(cur, co, parent))
            A = co.A.tocsr()  # rediscretised on the coarser leaves
            self.levels.append(Level("dg", A, n, cur.p, extract_diagonal_blocks(A, (cur.p + 1) ** dim)))
            cur, lv = co, lc
        P = cur.base_q1_prolongation()
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
        self.coarse_chol = sla.cho_factor(self.levels[-1].A.toarray())
