"""CPU oracle for the SuperDC rank-one conquer path.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The product library never does.
"""
from .oracle import (  # noqa: F401
    build, load, secular, loewner, bnorm, cauchy_apply, backward, validate,
    solve_batch, deflate, deflate_expand, deflated_eig, ST_UNSORTED, ST_ZERO, ST_NONFINITE, ST_RHO, ST_NOCONV,
)
