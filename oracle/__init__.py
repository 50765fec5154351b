"""Plain CPU FP64 reference of the block-preconditioned FGMRES solve.

TEST INFRASTRUCTURE ONLY.  This package is the parity oracle: only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
or run it.  The product path (the HIP library and its Python binding) never
touches it, and it shares no code with that path.

Every function follows a passage of Franceschini, Gazzola & Ferronato, "A
scalable preconditioning framework for stabilized contact mechanics with
hydraulically active fractures" (cited by section / equation / algorithm),
or, where the paper is silent (the multigrid details, the Krylov
bookkeeping), a published method named in the docstring.  Sparse products,
dense LU and sparse direct solves come from NumPy / SciPy; nothing is
blocked, fused or reordered beyond what the cited definition states.
"""
from .hashing import hash32, hash_unit
from .blocks import (bdiag_inv, bdiag_apply, bdiag_matrix, schur1,
                     schur_tpu, fixed_stress, s1_node_pattern)
from .amg import AMGOptions, Hierarchy, build_hierarchy, mis2_aggregate
from .precond import BlockPrecond
from .fgmres import fgmres
from . import adjoint

__all__ = ["hash32", "hash_unit", "bdiag_inv", "bdiag_apply", "bdiag_matrix",
           "schur1", "schur_tpu", "fixed_stress", "s1_node_pattern",
           "AMGOptions", "Hierarchy", "build_hierarchy", "mis2_aggregate",
           "BlockPrecond", "fgmres", "adjoint"]
