"""Oracle for the H*v hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow CPU reference (gcc-built C for the row-wise H*v, numpy/scipy for
the iterative methods). Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import it. It shares no code with the HIP library.
"""
from . import core  # noqa: F401
