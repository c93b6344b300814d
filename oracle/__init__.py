"""CPU oracle for the SymFT sampling stage.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU library.  See
``symft_oracle.c`` (full tableau + explicit FP64 active vector) and
``dense.py`` (plain state-vector brute force for small circuits).
"""
from .oracle import OracleCircuit, build, philox, rmeas_bit, active_u, gap_table, conjugate  # noqa: F401
from .counts import count_flags  # noqa: F401
