"""Plain FP64 CPU oracle for the sparsification A = U S V^T of an H^2 matrix.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product (the HIP
library and its Python binding) never does, and shares no code with it.

Modules:
  tree         cluster tree, block cluster tree, admissibility (Section 4.1)
  h2           Chebyshev H^2 construction, recompression, dense form, matvec
  householder  Householder QR with square Q (Section 4.2, LAPACK convention)
  sparsify     the level sweep producing Q_t, S and the pattern (Sections 2, 4)
  solve        U^T b / V y, block ILU(0) of S, iterative refinement (eq. sp0)

Parity status: every function is pinned by tests under tests/ against the
paper's identities (orthogonality, exactness U S V^T = A_H2, symmetry and
spectrum of S, sizes), closed-form special cases, brute force on tiny
inputs and library routines (LAPACK QR, dense LU), except the recompression
details (singular-vector choice inside the truncated subspace), which are
basis-dependent and pinned only through the basis-independent H^2 matrix.
"""

from .tree import (ClusterTree, BlockTree, build_cluster_tree, build_block_tree,
                   farfield_nonempty, admissible, tree_depth)
from .h2 import EXP, IFMM, H2Matrix, build_h2, kernel_block, close_block
from .householder import householder_qr
from .sparsify import (Sparsified, sparsify, apply_ut, apply_v, dense_s, dense_u,
                       pattern_predicate, cluster_sizes)
from .solve import (BlockILU0, dense_lu_solver, refine, rel_residual,
                    conjugate_gradient, elimination_order, elimination_colours,
                    block_fill, filled)
from .precond import BlockILUT, SymBlockILUT, gmres

__all__ = [
    "ClusterTree", "BlockTree", "build_cluster_tree", "build_block_tree",
    "farfield_nonempty", "admissible", "tree_depth", "H2Matrix", "build_h2",
    "EXP", "IFMM", "kernel_block", "close_block", "householder_qr", "Sparsified", "sparsify",
    "apply_ut", "apply_v", "dense_s", "dense_u", "pattern_predicate",
    "cluster_sizes", "BlockILU0", "dense_lu_solver", "refine", "rel_residual",
    "conjugate_gradient", "elimination_order", "elimination_colours",
    "block_fill", "filled", "BlockILUT", "SymBlockILUT", "gmres",
]
