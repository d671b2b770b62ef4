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
