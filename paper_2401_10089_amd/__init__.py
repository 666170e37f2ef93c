"""MI355X (gfx950) matrix logarithm: inverse scaling and squaring with the
computation-graph polynomials of Jarlebring, Sastre and Ibanez (arXiv 2401.10089).

All computation happens in the HIP library ``liblogm.so`` (C ABI in
``include/logm.h``); this package only marshals arguments.
"""

from ._binding import (  # noqa: F401
    EXPORTS,
    BatchPlan,
    autotune,
    autotune_batched,
    set_batched_split,
    balance,
    logm_batched,
    LIB_PATH,
    STATUS,
    LibraryNotBuilt,
    LogmError,
    default_opts,
    gemm,
    inverse,
    load_library,
    logm,
    logm_autograd,
    logm_backward,
    logm_backward_taped,
    logm_forward_taped,
    logm_noalloc,
    NOALLOC_MAX_N,
    Tape,
    backward_workspace_size,
    normest,
    poly,
    profile_enable,
    profile_get,
    profile_reset,
    scheme,
    sqrtm,
    strerror,
    version,
    workspace_size,
)
