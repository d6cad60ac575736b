"""CPU oracle for the fast directional Helmholtz matvec (Of & Watschinger).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy
implementation of the method, written from the paper to check the GPU
library against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never calls it and shares
no code with it (no kernels, tables, constants or helpers).

Layout, following the paper:

* ``tree``          Sect. 2.1, Alg. 1  -- uniform box cluster trees
* ``partition``     Sect. 2.2 Def. (A1)-(A3), Sect. 2.3 Alg. 2 -- block tree
* ``directions``    Sect. 2.4 Alg. 3, Def. of dir maps, Def. of active and
                    inherited directions
* ``interpolation`` Sect. 2.2 (Chebyshev interpolation, coupling matrices),
                    Sect. 2.5 and 2.7 (transfer matrices)
* ``fdmvm``         Sect. 2.6 Alg. 4 -- the matvec, plus a row-sampled variant
* ``dense``         Sect. 1 -- the dense product, for reference
* ``emulate``       reduced-precision emulation of the M2L step, used to fix
                    the tolerance of the mixed-precision GPU path
* ``lowrank``       Sect. 2.7 -- coupling matrices compressed by adaptive
                    cross approximation (matvec option ``m2l="aca:<eps>"``)

Readings of points the paper leaves open (node formula, child and face
ordering, tie-breaks, tree depth, high-frequency level rule) are listed in the
module that applies them.

Parity status: every function is pinned by a test against something other
than itself (closed forms, invariants, the paper's Table 1, brute force) except
the absolute approximation error at the workloads, which the paper does not
bound ("parity unpinned": reported only).
"""
from .tree import BoxTree, build_box_tree
from .partition import ETA2, admissible, block_tree, BlockTree
from .directions import (TAU_HF, high_frequency_level, DirectionSets,
                         active_directions)
from .interpolation import (chebyshev_nodes, lagrange_1d, multi_indices,
                            interpolation_rows, transfer_reference,
                            coupling_matrix, helmholtz)
from .fdmvm import Plan, build, matvec, sample_rows, structure
from .dense import dense_matvec, dense_rows
from .lowrank import aca, aca_dense

__all__ = [
    "BoxTree", "build_box_tree", "ETA2", "admissible", "block_tree",
    "BlockTree", "TAU_HF", "high_frequency_level", "DirectionSets",
    "active_directions", "chebyshev_nodes", "lagrange_1d", "multi_indices",
    "interpolation_rows", "transfer_reference", "coupling_matrix",
    "helmholtz", "Plan", "build", "matvec", "sample_rows", "structure",
    "dense_matvec", "dense_rows",
]
