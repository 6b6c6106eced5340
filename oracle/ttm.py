"""TTM-chain through the Kronecker reformulation (oracle; test infrastructure only).

Section 3, "Reformulation" (eq. 1) and Appendix A: the mode-n penultimate
matrix Z_(n) = T x_{j != n} F_j^T has one row per mode-n index l, and

    Z_(n)[l, :] = sum over elements e of slice l of  val(e) * Kron_n(e),

where Kron_n(e) is the Kronecker (outer) product of the factor rows
F_j[l_j(e), :] for j != n, vectorised lexicographically with the first
remaining mode fastest (position sum_j c_j * prod_{i<j} K_i over the remaining
modes).  The appendix lists the first row as coming from F_n; it is F_1 (the
product runs over j != n).

Everything here is FP64.
"""
from __future__ import annotations

import numpy as np


def kron_rows(factors, idx, n, elems):
    """Kron_n(e) for the elements ``elems`` (array of element indices): an
    (len(elems), prod_{j != n} K_j) FP64 matrix, first remaining mode fastest."""
    kr = np.ones((len(elems), 1), np.float64)
    for j in range(len(factors)):
        if j == n:
            continue
        rows = np.asarray(factors[j], np.float64)[np.asarray(idx[j])[elems]]   # (e, K_j)
        # new[c_prev + prev * c_j] = kr[c_prev] * rows[c_j]  (earlier modes fastest)
        kr = (rows[:, :, None] * kr[:, None, :]).reshape(len(elems), -1)
    return kr


def ttm_chain(idx, vals, factors, n, dims, chunk=1 << 16):
    """Full Z_(n) (dims[n] x Khat_n) by eq. 1, FP64."""
    vals = np.asarray(vals, np.float64)
    m = vals.shape[0]
    Khat = int(np.prod([np.asarray(f).shape[1] for j, f in enumerate(factors) if j != n]))
    Y = np.zeros((int(dims[n]), Khat), np.float64)
    rows_n = np.asarray(idx[n])
    for a in range(0, m, chunk):
        e = np.arange(a, min(a + chunk, m))
        contr = vals[e, None] * kron_rows(factors, idx, n, e)
        np.add.at(Y, rows_n[e], contr)
    return Y


def ttm_chain_rows(idx, vals, factors, n, slice_ids, chunk=1 << 16):
    """Rows Z_(n)[l, :] for the requested slice ids only (FP64): the elements
    of each requested slice, summed by eq. 1."""
    slice_ids = np.asarray(slice_ids, np.int64)
    rows_n = np.asarray(idx[n], np.int64)
    sel = np.flatnonzero(np.isin(rows_n, slice_ids))
    Khat = int(np.prod([np.asarray(f).shape[1] for j, f in enumerate(factors) if j != n]))
    Y = np.zeros((len(slice_ids), Khat), np.float64)
    srt = np.argsort(slice_ids, kind="stable")
    target = srt[np.searchsorted(slice_ids[srt], rows_n[sel])]
    vals = np.asarray(vals, np.float64)
    for a in range(0, sel.size, chunk):
        e = sel[a:a + chunk]
        contr = vals[e, None] * kron_rows(factors, idx, n, e)
        np.add.at(Y, target[a:a + chunk], contr)
    return Y


def nonempty_slices(idx_n, L_n):
    """Ascending ids of the mode-n slices holding at least one element."""
    return np.flatnonzero(np.bincount(np.asarray(idx_n, np.int64), minlength=L_n) > 0)


# ---------------------------------------------------------------------------------------------
# Dense definitions used to pin the reformulation (Section 2.1: unfolding, TTM).
# ---------------------------------------------------------------------------------------------

def dense(idx, vals, dims):
    """Dense FP64 tensor from coalesced COO."""
    T = np.zeros(tuple(int(d) for d in dims), np.float64)
    np.add.at(T, tuple(np.asarray(i, np.int64) for i in idx), np.asarray(vals, np.float64))
    return T


def unfold(T, n):
    """Mode-n unfolding T_(n): L_n x prod_{j != n} L_j with the fiber
    <l_1..l_{n-1}, l_{n+1}..l_N> in column sum_{j != n} l_j prod_{i != n, i < j} L_i
    (0-based; the first remaining mode varies fastest)."""
    Tn = np.moveaxis(T, n, 0)
    return Tn.reshape(T.shape[n], -1, order="F")


def ttm(T, A, n):
    """Mode-n TTM Z = T x_n A, realised as A @ T_(n) (Section 2.1)."""
    Zn = np.asarray(A, np.float64) @ unfold(T, n)
    shape = list(T.shape)
    shape[n] = Zn.shape[0]
    # fold back: inverse of unfold()
    moved = Zn.reshape([shape[n]] + [shape[j] for j in range(T.ndim) if j != n], order="F")
    return np.moveaxis(moved, 0, n)
