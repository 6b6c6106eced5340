"""Sparse HOOI Tucker decomposition on one MI355X (gfx950).

The hot path of Chakaravarthy et al., "On Optimizing Distributed Tucker
Decomposition for Sparse Tensors" (arXiv 1804.09494) as a HIP library behind a
C ABI (include/tucker_hip.h): per-mode sparse TTM-chain through the Kronecker
reformulation, Lite partition of the elements over workgroups, Gram on the
matrix cores, FP64 eigensolve and CholeskyQR2, core and fit, and the adjoint of
a Tucker-completion loss.  This package holds the build script and a thin
ctypes binding; every step runs in the library.
"""
from .api import TuckerContext, TuckerError  # noqa: F401

try:
    from .api import TuckerEval  # noqa: F401
except ImportError:  # torch missing
    pass
