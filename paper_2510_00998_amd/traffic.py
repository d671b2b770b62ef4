"""Algorithmic memory traffic of the smoother (host-side bookkeeping).

The paper's per-cell access counts (Section 4.1, "Reduction in memory
traffic", Table tab:memory_references) and the exact byte counts of one
launch of each kernel of this library, used as the numerator of the HBM
roofline.
"""
from __future__ import annotations


def words_vanilla(d: int, p: int) -> int:
    """Algorithm 1 (vanilla block-Jacobi): (2d+5)(p+1)^d accesses per cell."""
    return (2 * d + 5) * (p + 1) ** d


def words_facet(d: int, p: int) -> int:
    """Algorithms 2/4 (facet variables): 3(p+1)^d + 7d(p+1)^(d-1)."""
    return 3 * (p + 1) ** d + 7 * d * (p + 1) ** (d - 1)


def words_facet_exit(d: int, p: int) -> int:
    """Facet variables with a dynamic exit criterion: 5(p+1)^d + 7d(p+1)^(d-1)."""
    return 5 * (p + 1) ** d + 7 * d * (p + 1) ** (d - 1)


def words_fused_sweep(d: int, p: int) -> int:
    """Per-cell words of this library's fused sweep in the large-mesh limit:
    read u, read b, write u, and per facet side two trace fields (value and
    normal derivative) written once and read once: 3(p+1)^d + 8d(p+1)^(d-1)."""
    return 3 * (p + 1) ** d + 8 * d * (p + 1) ** (d - 1)


def interior_facets(d: int, n: int) -> int:
    return d * n ** (d - 1) * (n - 1)


def sweep_bytes(d: int, n: int, p: int, itemsize: int, per_cell_kappa: bool = False,
                block_recompute: bool = False) -> int:
    """Exact algorithmic bytes of one fused sweep launch on the n^d mesh:
    3 cell vectors, plus 2 sides x 2 fields x (p+1)^(d-1) trace values per
    interior facet read once and written once (boundary facets carry no
    traces), plus per-cell eigendata d((p+1)^2 + (p+1)) and kappa when the
    coefficient varies per cell (kappa alone when the kernels rebuild the
    eigendata in each traversal)."""
    N = p + 1
    ncell = n ** d
    words = 3 * ncell * N ** d + interior_facets(d, n) * 2 * 2 * N ** (d - 1) * 2
    if per_cell_kappa:
        words += ncell * (1 if block_recompute else d * (N * N + N) + 1)
    return words * itemsize


def project_bytes(d: int, n: int, p: int, itemsize: int) -> int:
    """Read u, write both sides' traces of every interior facet."""
    N = p + 1
    return (n ** d * N ** d + interior_facets(d, n) * 2 * 2 * N ** (d - 1)) * itemsize


def apply_bytes(d: int, n: int, p: int, itemsize: int, per_cell_kappa: bool = False) -> int:
    """Read u, read the neighbour traces, write y."""
    N = p + 1
    ncell = n ** d
    words = 2 * ncell * N ** d + interior_facets(d, n) * 2 * 2 * N ** (d - 1)
    if per_cell_kappa:
        words += ncell * (d * (N * N + N) + 1)
    return words * itemsize


# ---------------------------------------------------------------------------
# Bytes of a whole V-cycle and of one outer iteration, kernel by kernel as
# the library runs them (the numerator of the time-to-solution roofline).

def _trace_words(d: int, n: int, N: int) -> int:
    """Trace values of every interior facet, both sides, both fields."""
    return interior_facets(d, n) * 2 * 2 * N ** (d - 1)


def _p_levels(p: int) -> list:
    out, q = [p], p // 2
    while q >= 2:
        out.append(q)
        q //= 2
    return out


def _q1_levels(n: int, coarsest_n: int = 4) -> list:
    """Cells per axis of the Q1 levels (factor 2; an odd count keeps its last
    vertex, so m -> ceil(m/2))."""
    out = [n]
    m = n
    while m > coarsest_n:
        m = (m + 1) // 2
        out.append(m)
    return out


def q1_cycle_bytes(d: int, n: int, itemsize: int, nu_pre: int = 2, nu_post: int = 2, coarsest_n: int = 4) -> int:
    """Q1 part of a V-cycle entered with a zero guess: per level point-Jacobi
    steps (3^d stencil coefficients, inverse diagonal, b, u in and out),
    residual, restriction and prolongation; the dense coarsest solve reads
    its inverse (FP64)."""
    ns = 3 ** d
    lv = _q1_levels(n, coarsest_n)
    total = 0
    for i, m in enumerate(lv):
        nv = (m - 1) ** d
        if i + 1 == len(lv):
            total += nv * nv * 8 + 2 * nv * itemsize
            break
        nvc = (lv[i + 1] - 1) ** d
        words = 0
        for k in range(nu_pre):
            words += nv * (ns + 2 + (0 if k == 0 else 1)) + nv  # st, dinv, b, [u]; write u
        words += nv * (ns + 2) + nv          # residual: st, u, b -> r
        words += nv + nvc                    # restriction
        words += nvc + 2 * nv                # prolongation: coarse u, fine u in/out
        words += nu_post * (nv * (ns + 3) + nv)
        total += words * itemsize
    return total


def vcycle_bytes(d: int, n: int, p: int, itemsize: int, nu_pre: int = 2, nu_post: int = 2,
                 coarsest_n: int = 4) -> int:
    """One V-cycle from a zero guess (the preconditioner application): on
    each DG level (p halved while >= 2) the first sweep reads b and writes u
    and traces, the next ones are full sweeps, then residual + restriction
    (u, b, neighbour traces in; coarse right-hand side out), the coarser
    levels, prolongation + projection (u and the coarse vector in; u and
    traces out) and the post-smoothing sweeps; then the Q1 levels.  The
    coarser levels run in the compute type (FP32 for 16-bit storage)."""
    degs = _p_levels(p)
    total = 0
    ncell = n ** d
    for li, q in enumerate(degs):
        isz = itemsize if li == 0 else max(itemsize, 4)
        N = q + 1
        nd = ncell * N ** d
        tw = _trace_words(d, n, N)
        if li + 1 < len(degs):
            ndc = ncell * (degs[li + 1] + 1) ** d
            csz = max(itemsize, 4)
            rest_out, prol_in = ndc * csz, ndc * csz
        else:
            csz = max(itemsize, 4)
            nct = ncell * 2 ** d  # corner contributions, then gathered to the Q1 vertices
            nv = (n - 1) ** d
            rest_out = nct * csz + (nct + nv) * csz
            prol_in = nct * csz
        b = 0
        for k in range(nu_pre):
            b += (2 * nd + tw) * isz if k == 0 else sweep_bytes(d, n, q, isz)
        b += (2 * nd + tw) * isz + rest_out
        b += (2 * nd + tw) * isz + prol_in
        b += nu_post * sweep_bytes(d, n, q, isz)
        total += b
    return total + q1_cycle_bytes(d, n, max(itemsize, 4), nu_pre, nu_post, coarsest_n)


def fcg_iteration_bytes(d: int, n: int, p: int, cycle_itemsize: int, nu_pre: int = 2, nu_post: int = 2,
                        coarsest_n: int = 4) -> int:
    """One flexible-CG iteration of hpmg_solve: the V-cycle z = M r in the
    cycle's storage type, the dots z.r and z.(r - r_old) (z, r, r_old), the
    projection of p = z + beta p (z, p in; p and its FP64 traces out), q = A p
    (p and traces in, q out) and the update of u and r (u, r, p, q in; u, r,
    r_old and the FP32 copy of r out)."""
    N = p + 1
    nd = n ** d * N ** d
    tw = _trace_words(d, n, N)
    zs = cycle_itemsize
    b = vcycle_bytes(d, n, p, cycle_itemsize, nu_pre, nu_post, coarsest_n)
    b += nd * (zs + 16)                      # dots
    b += nd * (zs + 16) + tw * 8             # p = z + beta p, traces of p
    b += (2 * nd + tw) * 8                   # q = A p
    b += nd * 32 + nd * 24 + nd * min(zs, 4)  # update of u, r
    return b


def adaptive_facet_counts(d: int, n: int, r: int, leaves) -> dict:
    """Facet bookkeeping of a spacetree leaf list (rows (level, x_0, ..)):
    cell-facet sides on the boundary, hanging interfaces (a coarse leaf's
    facet whose neighbour region is refined) and r^(d-1) cells per
    interface."""
    index = {tuple(int(v) for v in row) for row in leaves}
    bdy = 0
    nif = 0
    for row in leaves:
        lvl, x = int(row[0]), [int(v) for v in row[1:]]
        ext = n * r ** lvl
        for k in range(d):
            for s in (-1, 1):
                y = list(x)
                y[k] += s
                if not 0 <= y[k] < ext:
                    bdy += 1
                    continue
                if (lvl, *y) in index:
                    continue
                if lvl > 0 and (lvl - 1, *[v // r for v in y]) in index:
                    continue
                nif += 1
    return {"boundary_sides": bdy, "interfaces": nif, "cells_per_interface": r ** (d - 1)}


def adaptive_sweep_bytes(d: int, n: int, r: int, leaves, p: int, itemsize: int, counts: dict | None = None) -> int:
    """Algorithmic bytes of one fused sweep on an adaptive mesh (the sweep
    launch and the hanging-facet remap after it): 3 cell vectors; per
    non-boundary cell-facet side the neighbour-side traces read and the own
    traces written (2 fields x (p+1)^(d-1) values each); per hanging
    interface its m + 1 own-trace slots read and its m + 1 remap slots
    written (m = r^(d-1)); per cell the 2d neighbour-slot indices (4 bytes),
    the facet mask (2 bytes) and in 3D the h scale (one compute-type value)."""
    N = p + 1
    L = N ** (d - 1)
    c = counts or adaptive_facet_counts(d, n, r, leaves)
    ncell = len(leaves)
    sides = 2 * d * ncell - c["boundary_sides"]
    m = c["cells_per_interface"]
    words = 3 * ncell * N ** d + sides * 2 * L * 2 + c["interfaces"] * (m + 1) * 2 * L * 2
    meta = ncell * (4 * 2 * d + 2 + (itemsize if d == 3 else 0))
    return words * itemsize + meta
