"""Seeded synthetic inputs for the fractured-medium block system.

This package builds the 3x3 block Jacobian ``J = [A C1 Q1; C2 -H 0; Q2 0 T]``
of the stabilized contact / fracture-flow model (Sec. 2.2, eq. JacSys and
eq. block_def of Franceschini, Gazzola & Ferronato, "A scalable
preconditioning framework for stabilized contact mechanics with hydraulically
active fractures") on structured hexahedral meshes with mesh-aligned
fractures, together with right-hand sides and the fracture flow graph.

It is the *input* side only: it holds none of the preconditioner, multigrid
or Krylov arithmetic.  Both the HIP library (through its C ABI) and the CPU
reference in ``oracle/`` consume what it produces.
"""
from .problem import (BlockSystem, Fracture, build_system, assemble_T,
                      flow_loss, transmissibility_pairs, reference_stiffness)
from .configs import (make_config, CONFIGS, tiny_system, rhs_batch,
                      observations)

__all__ = ["BlockSystem", "Fracture", "build_system", "assemble_T",
           "flow_loss", "transmissibility_pairs", "reference_stiffness",
           "make_config", "CONFIGS", "tiny_system", "rhs_batch",
           "observations"]
