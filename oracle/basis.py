"""1D nodal bases and quadrature for the oracle (test infrastructure only).

Paper reference: Section 2.2.1 (volumetric DG spaces: tensor-product
Lagrange polynomials on Gauss-Lobatto or Gauss-Legendre nodes) and the
remark on block-matrix structure in Section 4.1 (Gauss-Lobatto basis: exact
mass matrices need more than p+1 Lobatto points, so the mass is not
diagonal).  All quadrature here is Gauss-Legendre and exact for the
polynomial degrees integrated.

Pinned by tests/test_oracle_basis.py (closed-form GLL nodes for p <= 4,
quadrature exactness, derivative identities).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes on [0, 1]: the endpoints plus the roots of
    P_p' (derivative of the Legendre polynomial of degree p), sorted."""
    if p < 1:
        raise ValueError("p >= 1 required")
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gl_nodes(p: int) -> np.ndarray:
    """Gauss-Legendre nodes on [0, 1] (p+1 of them)."""
    x, _ = npleg.leggauss(p + 1)
    return 0.5 * (x + 1.0)


def gauss_rule(nq: int):
    """nq-point Gauss-Legendre rule on [0, 1] (exact to degree 2nq-1)."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(nodes: np.ndarray, x: np.ndarray):
    """Values V[k, j] = l_j(x_k) and derivatives D[k, j] = l_j'(x_k) of the
    Lagrange polynomials through `nodes`, by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(nodes)
    V = np.ones((len(x), m))
    D = np.zeros((len(x), m))
    for j in range(m):
        for l in range(m):
            if l == j:
                continue
            V[:, j] *= (x - nodes[l]) / (nodes[j] - nodes[l])
        for l in range(m):
            if l == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[l]))
            for mm in range(m):
                if mm == j or mm == l:
                    continue
                term *= (x - nodes[mm]) / (nodes[j] - nodes[mm])
            D[:, j] += term
    return V, D


def ref_matrices_1d(p: int, nodes: np.ndarray | None = None):
    """Reference-interval matrices on [0, 1] for the degree-p nodal basis:
    mass M[i, j] = int l_i l_j, stiffness K[i, j] = int l_i' l_j', both by
    (p+1)-point Gauss (exact for degree 2p)."""
    if nodes is None:
        nodes = gll_nodes(p)
    xq, wq = gauss_rule(p + 1)
    V, D = lagrange_1d(nodes, xq)
    M = V.T @ (wq[:, None] * V)
    K = D.T @ (wq[:, None] * D)
    return M, K
