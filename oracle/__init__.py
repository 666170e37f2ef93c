"""Oracle for the inverse-scaling-and-squaring matrix logarithm.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything from this package: it is used by ``tests/``, by
``__graft_entry__.smoke()`` (to check one small GPU result) and by the CPU
baseline leg of ``bench.py``.  It shares no code with the HIP library.

The implementation is a plain, slow, fp64 (or complex128) NumPy transcription of
the method of Jarlebring, Sastre and Ibanez, "Polynomial approximations for the
matrix logarithm with computation graphs" (arXiv 2401.10089); see
``logm_oracle`` for the step-by-step citations.
"""

from .logm_oracle import (  # noqa: F401
    TABLE2,
    THETA_FIT,
    THETA_DEFAULT,
    SHIPPED_K,
    TABMIN_IM,
    UNIT_ROUNDOFF,
    OracleError,
    scheme_coefficients,
    eval_scheme,
    norm1,
    normest_power,
    db_sqrt,
    select_degree,
    logm,
    balance,
    logm_backward,
    frechet_block,
)
