"""MI355X-native fast-convolution filtered CP-OFDM (arXiv 2008.00672).

The compute lives in libfc.so (hand-written gfx950 HIP kernels behind a C ABI,
declared in include/fc.h). ``fc`` is a ctypes binding of that ABI; importing
this package does not load the library, the first call does, and it raises if
the library has not been built.
"""
from .fc import (Plan, Graph, FcError, lib, CONT_OLA, CONT_OLS, SYNC_OLA, SYNC_OLS,  # noqa: F401
                 OP_TX, OP_RX, OP_ADJ, OP_RXD, OP_TXG)


def fc_tx(plan, x, w):
    """Differentiable FC synthesis (see ``autograd``)."""
    from .autograd import fc_tx as _f
    return _f(plan, x, w)
