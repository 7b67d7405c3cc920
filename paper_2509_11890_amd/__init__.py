"""MI355X tensor-train interior-point library (Python binding).

A thin ctypes layer over ``libttipm.so`` (declared in ``include/ttipm.h``):
it only marshals arguments — device pointers of torch tensors, ranks, the
current HIP stream — into the C ABI.  Every computation runs in the library's
HIP kernels; if the library is missing the import of the binding fails.
"""
from .binding import (  # noqa: F401
    lib, LibraryMissing, TTError, TT_OK, TT_LEFT, TT_RIGHT, TT_TOL_ABS, TT_TOL_REL,
    TTIPM_MAXCUT, TTIPM_THETA, TTIPM_CC, TTIPM_GENERIC, TTIPM_F64, TTIPM_MIXED, TT_F64, TT_F32, TT_BF16,
    TT_SOLVE_AUTO, TT_SOLVE_DIRECT, TT_SOLVE_GMRES, TT_SOLVE_CHOLESKY, TT_PREC_NONE, TT_PREC_BJACOBI, TT_PREC_MLP,
    contract_interfaces, local_matvec, local_matvec_noalloc, local_solve, tt_round, tt_round_workspace, op_inner,
    ProjOp,
    LocalBlock, LocalOp,
    Params, Problem, State, ttipm_step, ttipm_solve, version, profile_start, profile_stop, MLP,
)
