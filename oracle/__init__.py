"""CPU oracle for the SIPG-DG hp-multigrid hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 definitions written from the paper (arXiv 2510.00998):
the interior-penalty bilinear form is assembled explicitly as a sparse
matrix (Section 2.3, eq. weak_form_IP) and every solver component is the
textbook operation on that matrix (block-Jacobi, Section 2.3.2 eq.
block-Jacobi-IP; coarse-grid correction and multiplicative multigrid,
Section 5, Algorithms CoarseGridCorrection / MGMult).

The same definitions on uniform meshes also exist as plain C++ with OpenMP
(`c/sipg_oracle.cpp`, loaded by `coracle.py`), pinned against this one and
timed as the CPU baseline.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  The HIP library
never calls it, and it shares no code with the HIP library.

Parity status of each function is stated in its docstring; functions pinned
by the CPU test-suite are listed in tests/test_oracle_*.py.
"""
from .basis import gll_nodes, gauss_rule, lagrange_1d, ref_matrices_1d  # noqa: F401
from .sipg import SIPG, q1_stiffness  # noqa: F401
from .mg import Hierarchy, HierarchyOptions  # noqa: F401
from . import manufactured  # noqa: F401
