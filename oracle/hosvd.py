"""HOSVD initialisation (oracle; test infrastructure only).

Section 1 ("HOOI Procedure") and Section 2.2: HOOI starts from a given
decomposition, found for instance by the higher-order SVD (the factor F_n is
the leading K_n left singular vectors of the mode-n unfolding T_(n)), or from
random factors.  The paper does not say how the HOSVD is computed.

Reading taken here (a randomized range finder): the unfolding T_(n) has
prod_{j != n} L_j columns, too many to touch, so it is multiplied by a test
matrix Omega_n = kron of sketch matrices Omega_j (L_j x s_j, caller-drawn),
and F_n is the leading K_n left singular vectors of T_(n) Omega_n.  That
product is Z_(n) of eq. 1 with the sketches in place of the factors, so the
TTM-chain computes it.  For a tensor of multilinear rank at most K and
sketches in general position the range of T_(n) Omega_n is the range of
T_(n), and the result is exactly the truncated HOSVD.

Everything here is FP64.
"""
from __future__ import annotations

import numpy as np

from . import hooi as _hooi
from . import ttm as _ttm


def hosvd_sketched(idx, vals, dims, sketches, ranks):
    """F_n = leading ranks[n] left singular vectors of T_(n) (kron_{j != n}
    sketches[j]), for every n (all modes from the sketches).  Returns
    (factors, sigmas)."""
    F, S = [], []
    for n in range(len(dims)):
        Z = _ttm.ttm_chain(idx, vals, sketches, n, dims)
        U, s, _ = _hooi.leading_left_singular_vectors(Z, ranks[n])
        F.append(U)
        S.append(s)
    return F, S


def hosvd_dense(T, ranks):
    """The truncated HOSVD of a dense tensor from its unfoldings (the
    definition): F_n = leading ranks[n] left singular vectors of T_(n)."""
    T = np.asarray(T, np.float64)
    out = []
    for n, K in enumerate(ranks):
        Tn = np.moveaxis(T, n, 0).reshape(T.shape[n], -1)
        U, s, _ = np.linalg.svd(Tn, full_matrices=False)
        out.append(U[:, :K])
    return out
