"""FP64 CPU oracle for sparse HOOI Tucker decomposition — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy code that states what the GPU library
computes, each function citing the passage of Chakaravarthy et al., "On
Optimizing Distributed Tucker Decomposition for Sparse Tensors" (arXiv
1804.09494) it follows.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark may import it; the library's product path never
does, and this package imports nothing from the library.

Modules
  coo         coalescing of the COO element list (Section 3, "Distributed Framework")
  lite        the Lite distribution scheme and the three metrics
              (Section 4 metrics 1-3, Section 6, Figure "Lite", Theorem 6.1)
  ttm         the TTM-chain through the Kronecker reformulation (eq. 1, Appendix A)
  hooi        SVD step, HOOI invocation, core and fit (Section 2.2, Figure "HOOI")
  hosvd       HOSVD initialisation through a Kronecker-sketched range finder
              (Section 1 "HOOI Procedure", Section 2.2)
  completion  Tucker-completion loss and its gradient (the differentiation form;
              not in the paper, plain calculus on the Tucker model of Section 2.2)

Conventions: coordinates are 0-based (the paper's are 1-based); unfoldings and
Kronecker vectors put the first remaining mode fastest (Section 2.1, Appendix
A); the core is stored first index fastest.

Parity status: every function is pinned by a test outside itself (dense
unfoldings with numpy.kron, brute force, the paper's worked Lite example,
Theorem 6.1's bounds, LAPACK, finite differences).  None is "parity unpinned".
"""
from . import coo, lite, ttm, hooi, hosvd, completion  # noqa: F401
