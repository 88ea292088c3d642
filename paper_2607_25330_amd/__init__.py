"""MI355X-native PSFD solver: HIP kernels behind a C ABI (libpsfd.so) and a thin binding."""

from .psfd import (  # noqa: F401
    PSFD_C128,
    PSFD_C64_BF16PC_REFINE64,
    PSFD_C64_REFINE64,
    Batch,
    Plan,
    PsfdError,
    PsfdLibraryMissing,
    lib,
    psfd_adjoint,
    psfd_apply,
    psfd_destroy,
    psfd_eps_grad,
    psfd_layout_eps,
    psfd_plan,
    psfd_plan_batch,
    psfd_precond,
    psfd_residual,
    psfd_rhs,
    psfd_solve,
    psfd_solve_batch,
)
