"""CPU oracle for affine-gap (Gotoh H/E/F) alignment and Nussinov folding.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark.  The GPU library never imports, links or
calls anything here, and this package imports nothing from the GPU library.
"""
from .alnref import (  # noqa: F401
    GLOBAL, LOCAL, EXTEND, FULL, BAND, XDROP, ZDROP,
    OK, UNREACHABLE, CIGAR_CAP, BAD_SYMBOL,
    OP_I, OP_D, OP_EQ, OP_X,
    align, align_batch, build, load,
)
from .foldref import fold, fold_batch, FOLD_DTYPE, NO_XDROP  # noqa: F401,E402
