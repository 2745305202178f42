"""MI355X-native central-moment discrete Boltzmann method (arXiv:2502.16818).

The method's step runs in hand-written HIP kernels for gfx950 behind the C
ABI of include/cdbm.h (libcdbm.so, built by ``paper_2502_16818_amd.build``).
This package holds the build script, the ctypes binding and the autograd
wrapper of the hand-written adjoint.
"""
from .cdbm import (  # noqa: F401
    BATCH_CONTIGUOUS, BATCH_ROW_PIECES, EXPORTS, FP64, MIXED, MIXED_COMP, PERIODIC, ZERO_GRADIENT,
    Batch,
    CdbmError, Params, Solver, load, make_params,
)
