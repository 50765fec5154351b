"""MI355X-native block-preconditioned FGMRES for stabilized contact mechanics
with hydraulically active fractures (t-u-p / t-p-u block preconditioners with
a smoothed-aggregation AMG inner solve), as a HIP library with a C ABI."""
from .fracprec import (Solver, FpcError, load_library, default_options,
                       solver_from_system, LIB_PATH, EXPORTS, STATUS)

__all__ = ["Solver", "FpcError", "load_library", "default_options",
           "solver_from_system", "LIB_PATH", "EXPORTS", "STATUS"]
