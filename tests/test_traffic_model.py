"""The per-cell access counts printed in the paper's Table
tab:memory_references (Section 4.1) reproduced by the traffic formulas."""
import os

import pytest

from paper_2510_00998_amd import traffic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "memory_references.txt")


def _rows():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        out[(int(parts[0]), parts[1])] = [float(x) for x in parts[2:]]
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_table_counts(d):
    rows = _rows()
    for i, p in enumerate(range(1, 11)):
        assert traffic.words_vanilla(d, p) == rows[(d, "vanilla")][i]
        assert traffic.words_facet(d, p) == rows[(d, "facet")][i]
        assert traffic.words_facet_exit(d, p) == rows[(d, "facet_exit")][i]
        r = traffic.words_vanilla(d, p) / traffic.words_facet(d, p)
        assert abs(r - rows[(d, "reduction")][i]) <= 0.0051
        r = traffic.words_vanilla(d, p) / traffic.words_facet_exit(d, p)
        assert abs(r - rows[(d, "reduction_exit")][i]) <= 0.0051


def test_exact_sweep_bytes_tends_to_per_cell_model():
    # interior cells dominate for large n: bytes/cell -> words_fused_sweep
    d, p, n = 3, 4, 400
    per_cell = traffic.sweep_bytes(d, n, p, 1) / n ** d
    assert abs(per_cell / traffic.words_fused_sweep(d, p) - 1) < 0.01
    # 32^3, Q4, FP64: 3 * 4.096e6 * 8 B of cell data + 95232 facets * 200 words * 8 B
    assert traffic.sweep_bytes(3, 32, 4, 8) == (3 * 32 ** 3 * 125 + 3 * 32 * 32 * 31 * 200) * 8
