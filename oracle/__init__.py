"""Plain FP64 CPU oracle for the recursively preconditioned hierarchical interpolative
factorization (test infrastructure only; see rhif_oracle for the rules on its use)."""
from .rhif_oracle import (  # noqa: F401
    NotSPDError,
    assemble_fd,
    fd_energy,
    dof_coords,
    num_levels,
    classify,
    closure_keys,
    chol,
    cpqr_id,
    factor,
    apply_inverse,
    apply_ginv,
    apply_ginv_t,
    apply_forward,
    estimate_ea,
    estimate_es,
    pcg,
    dense_solve,
    grad_log_a,
)
