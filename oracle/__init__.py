"""CPU oracle for P1 and P_k assembly.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    OP, STATUS, OracleError, build, lib_path, validate, assemble, assemble_rows,
    grad, element_matrix, assemble_lame, general_coef, assemble_general, boundary_mass, jvp, vjp, pk_ndfe, pk_alpha, pk_coeff, pk_mass, pk_mass_rows,
)
