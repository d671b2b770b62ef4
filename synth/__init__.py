"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the solver method itself: it only draws
random numbers and builds coefficient fields / right-hand-side vectors from
them.  Both sides (the CPU oracle and the HIP library) receive the arrays
produced here as plain data.

Random numbers come from splitmix64 (Steele, Lea, Flood: "Fast splittable
pseudorandom number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15,
then the published mix z ^= z>>30, *0xBF58476D1CE4E5B9, z ^= z>>27,
*0x94D049BB133111EB, z ^= z>>31.  Uniforms use the top 53 bits; normals use
the Box-Muller transform.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """Return `count` consecutive splitmix64 outputs for stream `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normal doubles by Box-Muller on pairs of uniforms."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m)
    u1 = 1.0 - u[0::2]  # in (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:count]


def n_cells(dim: int, n: int) -> int:
    return n ** dim


def cell_centres(dim: int, n: int) -> np.ndarray:
    """Cell centres of the uniform n^dim mesh of the unit box; cell index
    c = cx + n*cy (+ n^2*cz), shape (n^dim, dim)."""
    g = (np.arange(n) + 0.5) / n
    if dim == 2:
        cy, cx = np.meshgrid(g, g, indexing="ij")
        return np.stack([cx.ravel(), cy.ravel()], axis=1)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)


def kappa_log_uniform(dim: int, n: int, seed: int, lo: float = 1e-2, hi: float = 1e2) -> np.ndarray:
    """Piecewise-constant coefficient, log-uniform in [lo, hi], iid per cell."""
    u = uniform(seed, n_cells(dim, n))
    return np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)


def kappa_log_normal(dim: int, n: int, seed: int, sigma_log: float = 2.0,
                     corr_len: float = 0.1, modes: int = 1024) -> np.ndarray:
    """Piecewise-constant log-normal coefficient kappa_K = exp(sigma_log*g(x_K)).

    g is a random-Fourier-feature sample of a unit-variance Gaussian field with
    squared-exponential covariance of length `corr_len`:
    g(x) = sqrt(2/M) sum_m cos(w_m . x + phi_m), w_m ~ N(0, corr_len^-2 I),
    phi_m ~ U[0, 2pi), evaluated at the cell centres.
    """
    w = normal(seed, modes * dim).reshape(modes, dim) / corr_len
    phi = 2.0 * math.pi * uniform(seed + 1, modes)
    x = cell_centres(dim, n)
    g = np.zeros(x.shape[0])
    chunk = 65536
    for s in range(0, x.shape[0], chunk):
        g[s:s + chunk] = np.cos(x[s:s + chunk] @ w.T + phi).sum(axis=1)
    g *= math.sqrt(2.0 / modes)
    return np.exp(sigma_log * g)


def random_rhs(ndof: int, seed: int) -> np.ndarray:
    """Right-hand-side vector with iid N(0,1) entries."""
    return normal(seed, ndof)


def random_vector(ndof: int, seed: int) -> np.ndarray:
    """Test vector with iid U(-1, 1) entries."""
    return 2.0 * uniform(seed, ndof) - 1.0


def batched_problem_list(count: int = 64, seed: int = 1004, nmin: int = 8, nmax: int = 48,
                         pmin: int = 1, pmax: int = 5):
    """Mesh sizes n_j ~ U{nmin..nmax} and degrees p_j ~ U{pmin..pmax}."""
    u = uniform(seed, 2 * count)
    ns = nmin + np.minimum((u[0::2] * (nmax - nmin + 1)).astype(int), nmax - nmin)
    ps = pmin + np.minimum((u[1::2] * (pmax - pmin + 1)).astype(int), pmax - pmin)
    return [(int(a), int(b)) for a, b in zip(ns, ps)]


def batched_rhs_seed(base: int, problem: int, rhs: int) -> int:
    """Stream id of right-hand side `rhs` of problem `problem`."""
    return base * (1 << 32) + 4 * problem + rhs


# ---------------------------------------------------------------- spacetrees
# Leaf lists of hierarchical Cartesian meshes: n^dim base cells (level 0),
# a cell at level l split into r^dim children of width 1/(n r^(l+1)).  A
# leaf is (level, x_0, .., x_{dim-1}) with integer coordinates at its level.
# Mesh generation only: which cells are refined, then the facet balance
# (facet neighbours at most one level apart), then the depth-first order
# (base cells x fastest, children x fastest within their parent).

def _children(node, dim, r):
    lvl, x = node
    out = []
    for m in range(r ** dim):
        off = [(m // r ** k) % r for k in range(dim)]
        out.append((lvl + 1, tuple(r * x[k] + off[k] for k in range(dim))))
    return out


def _leaves_of(dim, n, r, refined):
    """Depth-first leaf list of the tree whose refined nodes are `refined`."""
    leaves = []

    def visit(node):
        if node in refined:
            for ch in _children(node, dim, r):
                visit(ch)
        else:
            leaves.append((node[0],) + node[1])

    for b in range(n ** dim):
        visit((0, tuple((b // n ** k) % n for k in range(dim))))
    return np.array(leaves, dtype=np.int64).reshape(-1, 1 + dim)


def _balance(dim, n, r, refined):
    """Refine leaves until every facet neighbour of a leaf at level l is a
    leaf at level l-1, l or l+1."""
    refined = set(refined)
    while True:
        leaves = _leaves_of(dim, n, r, refined)
        add = []
        for row in leaves:
            lvl, x = int(row[0]), tuple(int(v) for v in row[1:])
            ext = n * r ** lvl
            for k in range(dim):
                for s in (-1, 1):
                    y = list(x)
                    y[k] += s
                    if not 0 <= y[k] < ext:
                        continue
                    nb = (lvl, tuple(y))
                    if nb not in refined:
                        continue
                    # children of the neighbour that touch the shared facet
                    for ch in _children(nb, dim, r):
                        if ch[1][k] == (r * y[k] + (0 if s > 0 else r - 1)) and ch in refined:
                            add.append((lvl, x))
                            break
        add = set(add) - refined
        if not add:
            return leaves
        refined |= add


def spacetree_leaves(dim: int, n: int, r: int, refine, max_level: int) -> np.ndarray:
    """Leaves of the balanced spacetree in which a node (level l, coordinates
    x) with l < max_level is refined when refine(l, lower corner, width) is
    true; shape (nleaf, 1 + dim), rows (level, x_0, ..)."""
    refined = set()
    frontier = [(0, tuple((b // n ** k) % n for k in range(dim))) for b in range(n ** dim)]
    while frontier:
        nxt = []
        for node in frontier:
            lvl, x = node
            h = 1.0 / (n * r ** lvl)
            if lvl < max_level and refine(lvl, np.array(x, dtype=np.float64) * h, h):
                refined.add(node)
                nxt.extend(_children(node, dim, r))
        frontier = nxt
    return _balance(dim, n, r, refined)


def ball_refinement(centres, radii):
    """Refinement test: refine the cells that meet one of the balls."""
    centres = [np.asarray(c, dtype=np.float64) for c in centres]

    def refine(lvl, lo, h):
        for c, rad in zip(centres, radii):
            nearest = np.clip(c[: len(lo)], lo, lo + h)
            if np.sum((nearest - c[: len(lo)]) ** 2) <= rad * rad:
                return True
        return False

    return refine


def random_refinement(seed: int, frac: float):
    """Refinement test: refine a cell with probability frac (one uniform per
    cell, drawn from stream seed at an index hashed from level and corner)."""
    def refine(lvl, lo, h):
        key = int(lvl) * 1000003 + int(round(lo[0] / h)) * 7919 + int(round(lo[1] / h)) * 104729
        if len(lo) > 2:
            key += int(round(lo[2] / h)) * 1299709
        return float(uniform(seed * (1 << 20) + key, 1)[0]) < frac

    return refine


def leaf_centres(dim: int, n: int, r: int, leaves: np.ndarray) -> np.ndarray:
    """Centres of the leaves (nleaf, dim)."""
    h = 1.0 / (n * np.power(float(r), leaves[:, 0]))
    return (leaves[:, 1:1 + dim] + 0.5) * h[:, None]
