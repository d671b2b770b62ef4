"""Assembled SIPG operator for the oracle (test infrastructure only).

Discretisation (paper Section 2, with these readings where the paper is silent
or ambiguous):

* mesh: unit box [0,1]^d, n cells per axis, h = 1/n (Section 2.1, uniform
  instead of 3-partitioned); cell index c = cx + n*cy (+ n^2*cz);
* basis: tensor-product Lagrange on Gauss-Lobatto nodes, local index
  i = a + N*b (+ N^2*c), N = p+1, x fastest (Section 2.2.1);
* bilinear form: eq. weak_form_IP with theta = -1 (symmetric interior
  penalty), a piecewise-constant coefficient kappa_K and harmonic face
  coefficient kappa_F = 2 k- k+ / (k- + k+) in both flux and penalty terms;
  jump [v] = v- - v+, average {v} = (v- + v+)/2, n_F along +axis on interior
  facets and outward on boundary facets (Section 2.3.1);
* penalty: gamma_F = sigma = sigma0 (p_pen+1)^2 / h on interior facets and
  2 sigma on boundary facets (constant gamma-bar = 2 sigma, Section 4.1 after
  eq. weak_form_IP_facet_spaces), sigma0 = 2;
* all integrals by tensor Gauss-Legendre quadrature exact for the integrand.

The matrix is the plain definition a(phi_j, phi_i) written out by quadrature;
it shares nothing with the matrix-free HIP operator.  Pinned by
tests/test_oracle_sipg.py (symmetry, positive definiteness, annihilation of
global linears away from the boundary, exact reproduction of polynomial
solutions, Galerkin identities, manufactured-solution convergence rates).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import gauss_rule, gll_nodes, gl_nodes, lagrange_1d


def _kron_dims(mats):
    """Tensor-product evaluation matrix with x fastest: mats = [Mx, My(, Mz)]."""
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(m, out)
    return out


class SIPG:
    """Symmetric interior penalty DG discretisation of -div(kappa grad u) = f
    with homogeneous Dirichlet conditions (paper eq. weak_form_IP)."""

    def __init__(self, dim: int, n: int, p: int, kappa=None, p_penalty: int | None = None,
                 sigma0: float = 2.0, basis: str = "gll"):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim, self.n, self.p = dim, n, p
        self.N = p + 1
        self.nd = self.N ** dim
        self.ncell = n ** dim
        self.ndof = self.ncell * self.nd
        self.h = 1.0 / n
        if kappa is None:
            kappa = 1.0
        kappa = np.asarray(kappa, dtype=np.float64)
        if kappa.ndim == 0:
            kappa = np.full(self.ncell, float(kappa))
        if kappa.shape != (self.ncell,) or not np.all(kappa > 0):
            raise ValueError("kappa must be positive, one value per cell")
        self.kappa = kappa
        self.p_penalty = p if p_penalty is None else p_penalty
        self.sigma = sigma0 * (self.p_penalty + 1) ** 2 / self.h
        self.basis = basis
        self.nodes1d = gll_nodes(p) if basis == "gll" else gl_nodes(p)
        self._reference_blocks()
        self._A = None

    # ------------------------------------------------------------------ geometry
    def strides(self):
        return [1, self.n, self.n * self.n][: self.dim]

    def cell_index_coords(self):
        """(ncell, dim) integer cell coordinates."""
        c = np.arange(self.ncell)
        out = []
        for k in range(self.dim):
            out.append((c // (self.n ** k)) % self.n)
        return np.stack(out, axis=1)

    def dof_coords(self):
        """Physical coordinates of every nodal degree of freedom (ndof, dim)."""
        cc = self.cell_index_coords().astype(np.float64)
        xi = self.nodes1d
        loc = []
        for k in range(self.dim):
            idx = (np.arange(self.nd) // (self.N ** k)) % self.N
            loc.append(xi[idx])
        loc = np.stack(loc, axis=1)  # (nd, dim)
        X = (cc[:, None, :] + loc[None, :, :]) * self.h
        return X.reshape(-1, self.dim)

    # --------------------------------------------------------- reference blocks
    def _reference_blocks(self):
        d, N, h = self.dim, self.N, self.h
        xq, wq = gauss_rule(N)
        V, D = lagrange_1d(self.nodes1d, xq)
        e0, d0 = lagrange_1d(self.nodes1d, np.array([0.0]))
        e1, d1 = lagrange_1d(self.nodes1d, np.array([1.0]))
        self._V1, self._D1, self._wq = V, D, wq
        # volume: h^(d-2) sum_k int grad_k phi_i grad_k phi_j on the unit cell
        W = _kron_dims([np.diag(wq)] * d)
        Kv = np.zeros((self.nd, self.nd))
        for k in range(d):
            G = _kron_dims([D if j == k else V for j in range(d)])
            Kv += G.T @ W @ G
        self.Kvol = h ** (d - 2) * Kv
        # faces normal to axis k.  "minus" cell sees the facet at xi_k = 1,
        # "plus" cell at xi_k = 0; n_F = +e_k; physical d/dx_k = (1/h) d/dxi_k.
        self.face_val = {}
        self.face_dn = {}
        self.face_w = None
        Wf = _kron_dims([np.diag(wq)] * (d - 1)) * h ** (d - 1)
        self.face_w = Wf
        for k in range(d):
            for side, (ev, dv) in (("minus", (e1, d1)), ("plus", (e0, d0))):
                self.face_val[(k, side)] = _kron_dims([ev if j == k else V for j in range(d)])
                self.face_dn[(k, side)] = _kron_dims([dv / h if j == k else V for j in range(d)])
        # interior facet blocks B[(k, Y, X)]: rows test functions of side Y,
        # columns trial functions of side X, without the kappa_F factor.
        sgn = {"minus": 1.0, "plus": -1.0}
        self.Bint = {}
        for k in range(d):
            for Y in ("minus", "plus"):
                for X in ("minus", "plus"):
                    VY, DY = self.face_val[(k, Y)], self.face_dn[(k, Y)]
                    VX, DX = self.face_val[(k, X)], self.face_dn[(k, X)]
                    # -<{d_n u}[v]> - <{d_n v}[u]> + sigma <[u][v]>
                    B = (-0.5 * sgn[Y] * VY.T @ Wf @ DX
                         - 0.5 * sgn[X] * DY.T @ Wf @ VX
                         + self.sigma * sgn[X] * sgn[Y] * VY.T @ Wf @ VX)
                    self.Bint[(k, Y, X)] = B
        # boundary facet blocks (without kappa_K): outward normal, penalty 2 sigma.
        # -<d_n u v> - <d_n v u> + 2 sigma <u v>
        self.Bbdy = {}
        for k in range(d):
            for side in (0, 1):
                if side == 1:
                    Vb, Db = self.face_val[(k, "minus")], self.face_dn[(k, "minus")]
                else:
                    Vb, Db = self.face_val[(k, "plus")], -self.face_dn[(k, "plus")]
                self.Bbdy[(k, side)] = (-Vb.T @ Wf @ Db - Db.T @ Wf @ Vb
                                        + 2.0 * self.sigma * Vb.T @ Wf @ Vb)

    # ------------------------------------------------------------------ assembly
    def diagonal_blocks(self):
        """Exact diagonal blocks A_{K<-K}, shape (ncell, nd, nd)."""
        d, n = self.dim, self.n
        cc = self.cell_index_coords()
        blocks = self.kappa[:, None, None] * self.Kvol[None]
        kap = self.kappa
        for k in range(d):
            s = self.strides()[k]
            for side in (0, 1):
                at_bdy = cc[:, k] == (0 if side == 0 else n - 1)
                cells = np.nonzero(at_bdy)[0]
                blocks[cells] += kap[cells, None, None] * self.Bbdy[(k, side)][None]
                cells = np.nonzero(~at_bdy)[0]
                nb = cells + (s if side == 1 else -s)
                kf = 2.0 * kap[cells] * kap[nb] / (kap[cells] + kap[nb])
                own = "minus" if side == 1 else "plus"
                blocks[cells] += kf[:, None, None] * self.Bint[(k, own, own)][None]
        return blocks

    def offdiagonal_blocks(self):
        """List of (row cell array, col cell array, blocks array)."""
        out = []
        cc = self.cell_index_coords()
        kap = self.kappa
        for k in range(self.dim):
            s = self.strides()[k]
            lo = np.nonzero(cc[:, k] < self.n - 1)[0]
            hi = lo + s
            kf = 2.0 * kap[lo] * kap[hi] / (kap[lo] + kap[hi])
            out.append((lo, hi, kf[:, None, None] * self.Bint[(k, "minus", "plus")][None]))
            out.append((hi, lo, kf[:, None, None] * self.Bint[(k, "plus", "minus")][None]))
        return out

    @property
    def A(self) -> sp.bsr_matrix:
        """The assembled operator as a block-sparse (BSR) matrix."""
        if self._A is None:
            self._A = self._assemble()
        return self._A

    def _assemble(self):
        nd, nc = self.nd, self.ncell
        rows = [np.arange(nc)]
        cols = [np.arange(nc)]
        data = [self.diagonal_blocks()]
        for r, c, b in self.offdiagonal_blocks():
            rows.append(r)
            cols.append(c)
            data.append(b)
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        data = np.concatenate(data)
        order = np.lexsort((cols, rows))
        rows, cols, data = rows[order], cols[order], data[order]
        indptr = np.zeros(nc + 1, dtype=np.int64)
        np.add.at(indptr, rows + 1, 1)
        indptr = np.cumsum(indptr)
        return sp.bsr_matrix((data, cols, indptr), shape=(nc * nd, nc * nd))

    def apply_rows(self, cells, u):
        """(A u) restricted to the block rows of `cells`, computed from the
        block row of each cell only (for sampled parity at large sizes)."""
        cells = np.asarray(cells)
        nd, n, d = self.nd, self.n, self.dim
        U = u.reshape(self.ncell, nd)
        cc = self.cell_index_coords()[cells]
        kap = self.kappa
        y = np.einsum("cij,cj->ci", self._diag_blocks_for(cells), U[cells])
        for k in range(d):
            s = self.strides()[k]
            for side in (0, 1):
                has = cc[:, k] != (0 if side == 0 else n - 1)
                sel = np.nonzero(has)[0]
                cs = cells[sel]
                nb = cs + (s if side == 1 else -s)
                kf = 2.0 * kap[cs] * kap[nb] / (kap[cs] + kap[nb])
                B = self.Bint[(k, "minus", "plus")] if side == 1 else self.Bint[(k, "plus", "minus")]
                y[sel] += kf[:, None] * (U[nb] @ B.T)
        return y

    def _diag_blocks_for(self, cells):
        cells = np.asarray(cells)
        d, n = self.dim, self.n
        cc = self.cell_index_coords()[cells]
        kap = self.kappa
        blocks = kap[cells, None, None] * self.Kvol[None]
        for k in range(d):
            s = self.strides()[k]
            for side in (0, 1):
                at_bdy = cc[:, k] == (0 if side == 0 else n - 1)
                idx = np.nonzero(at_bdy)[0]
                blocks[idx] += kap[cells[idx], None, None] * self.Bbdy[(k, side)][None]
                idx = np.nonzero(~at_bdy)[0]
                cs = cells[idx]
                nb = cs + (s if side == 1 else -s)
                kf = 2.0 * kap[cs] * kap[nb] / (kap[cs] + kap[nb])
                own = "minus" if side == 1 else "plus"
                blocks[idx] += kf[:, None, None] * self.Bint[(k, own, own)][None]
        return blocks

    # ---------------------------------------------------------------- load vector
    def load_vector(self, f, nq: int | None = None) -> np.ndarray:
        """b_i = int f phi_i by (p+3)-point Gauss per direction (eq. in
        Section 2.3.1, b(v) = (v f))."""
        d = self.dim
        if nq is None:
            nq = self.p + 3
        xq, wq = gauss_rule(nq)
        V, _ = lagrange_1d(self.nodes1d, xq)
        Phi = _kron_dims([V] * d)  # (nq^d, nd)
        wt = _kron_dims([wq[None, :]] * d).ravel() * self.h ** d
        loc = []
        for k in range(d):
            idx = (np.arange(nq ** d) // (nq ** k)) % nq
            loc.append(xq[idx])
        loc = np.stack(loc, axis=1)
        cc = self.cell_index_coords().astype(np.float64)
        b = np.empty((self.ncell, self.nd))
        chunk = max(1, 2_000_000 // (nq ** d))
        for s0 in range(0, self.ncell, chunk):
            X = (cc[s0:s0 + chunk, None, :] + loc[None]) * self.h
            fv = f(X.reshape(-1, d)).reshape(X.shape[0], -1)
            b[s0:s0 + chunk] = (fv * wt[None]) @ Phi
        return b.ravel()

    def interpolate(self, g) -> np.ndarray:
        """Nodal interpolant of g (its values at the degrees of freedom)."""
        return g(self.dof_coords())

    def l2_error(self, u, g, nq: int | None = None) -> float:
        """Continuous L2 norm of (u_h - g) by Gauss quadrature."""
        d = self.dim
        if nq is None:
            nq = self.p + 3
        xq, wq = gauss_rule(nq)
        V, _ = lagrange_1d(self.nodes1d, xq)
        Phi = _kron_dims([V] * d)
        wt = _kron_dims([wq[None, :]] * d).ravel() * self.h ** d
        loc = []
        for k in range(d):
            idx = (np.arange(nq ** d) // (nq ** k)) % nq
            loc.append(xq[idx])
        loc = np.stack(loc, axis=1)
        cc = self.cell_index_coords().astype(np.float64)
        X = (cc[:, None, :] + loc[None]) * self.h
        uq = u.reshape(self.ncell, self.nd) @ Phi.T
        gq = g(X.reshape(-1, d)).reshape(self.ncell, -1)
        return float(np.sqrt(np.sum((uq - gq) ** 2 * wt[None])))


def q1_stiffness(dim: int, n: int, kappa=None) -> sp.csr_matrix:
    """Continuous Q1 finite-element stiffness sum_K kappa_K (grad phi_i,
    grad phi_j)_K on the interior vertices of the uniform n^d mesh (paper
    eq. weak_form_cg), assembled from its own element integrals."""
    h = 1.0 / n
    ncell = n ** dim
    if kappa is None:
        kappa = np.ones(ncell)
    kappa = np.asarray(kappa, dtype=np.float64)
    if kappa.ndim == 0:
        kappa = np.full(ncell, float(kappa))
    xq, wq = gauss_rule(2)
    # 1D hat pieces on the reference interval: phi_0 = 1 - x, phi_1 = x
    V = np.stack([1.0 - xq, xq], axis=1)
    D = np.stack([-np.ones_like(xq), np.ones_like(xq)], axis=1)
    W = _kron_dims([np.diag(wq)] * dim)
    Ke = np.zeros((2 ** dim, 2 ** dim))
    for k in range(dim):
        G = _kron_dims([D if j == k else V for j in range(dim)])
        Ke += G.T @ W @ G
    Ke *= h ** (dim - 2)
    nv = n - 1
    rows, cols, vals = [], [], []
    for c in range(ncell):
        cc = [(c // n ** k) % n for k in range(dim)]
        gidx = []
        for loc in range(2 ** dim):
            v = [cc[k] + ((loc >> k) & 1) for k in range(dim)]
            if any(vk == 0 or vk == n for vk in v):
                gidx.append(-1)
            else:
                gidx.append(sum((v[k] - 1) * nv ** k for k in range(dim)))
        for i in range(2 ** dim):
            if gidx[i] < 0:
                continue
            for j in range(2 ** dim):
                if gidx[j] < 0:
                    continue
                rows.append(gidx[i])
                cols.append(gidx[j])
                vals.append(kappa[c] * Ke[i, j])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nv ** dim, nv ** dim))
