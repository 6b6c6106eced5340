"""SVD step, HOOI invocation, core and fit (oracle; test infrastructure only).

Section 2.2 ("HOOI Procedure") and its figure: one invocation refines a
decomposition {G; F_1..F_N} mode by mode.  For mode n it forms the penultimate
matrix Z_(n) = (T x_{j != n} F_j^T)_(n) (eq. 1) and takes the leading K_n left
singular vectors of Z_(n) as the new F_n.  The core G = T x_1 F_1^T ... x_N F_N^T
is needed only once, after the invocations.

Readings (the paper is silent or ambiguous):
  * sweep order: Gauss-Seidel by default (mode n uses the factors already
    refined in this invocation for modes < n), the textbook HOOI that makes the
    fit non-decreasing; Jacobi (every mode uses the invocation's input
    factors, as the figure literally reads) is available as an option;
  * fit = 1 - sqrt(max(0, ||T||^2 - ||G||^2)) / ||T|| (Kolda-Bader form; the
    paper defines none);
  * SVD route: Householder QR of Z, then the SVD of the small R factor
    (LAPACK through numpy); deliberately not the Gram route the GPU takes;
  * rank deficiency (fewer than K_n nonzero singular values): the missing
    columns are completed by Gram-Schmidt of the lowest-index unit vectors not
    yet spanned; such columns are not unique and are not compared.
"""
from __future__ import annotations

import numpy as np

from . import ttm as _ttm


def leading_left_singular_vectors(Z, K, rel_zero=None):
    """(U, sigma, n_valid): the leading K left singular vectors of Z (FP64).

    n_valid = number of columns backed by a singular value above the zero
    threshold; columns past it come from the completion rule."""
    Z = np.asarray(Z, np.float64)
    rows, cols = Z.shape
    if rows >= cols:
        Q, R = np.linalg.qr(Z)
        Ur, s, _ = np.linalg.svd(R)
        U = Q @ Ur
    else:
        U, s, _ = np.linalg.svd(Z, full_matrices=False)
    if rel_zero is None:
        rel_zero = max(rows, cols) * np.finfo(np.float64).eps
    smax = s[0] if s.size else 0.0
    n_valid = int(np.sum(s[:K] > rel_zero * smax)) if smax > 0 else 0
    Uk = np.zeros((rows, K), np.float64)
    Uk[:, :n_valid] = U[:, :n_valid]
    sig = np.zeros(K)
    sig[:min(K, s.size)] = s[:K]
    col = n_valid
    i = 0
    while col < K:
        if i >= rows:
            raise ValueError("K exceeds the number of rows")
        v = np.zeros(rows)
        v[i] = 1.0
        for _ in range(2):
            v -= Uk[:, :col] @ (Uk[:, :col].T @ v)
        nv = np.linalg.norm(v)
        if nv > 0.5:
            Uk[:, col] = v / nv
            col += 1
        i += 1
    return Uk, sig, n_valid


def core(idx, vals, factors):
    """G[c_1..c_N] = sum_e val(e) prod_n F_n[l_n(e), c_n]  (the definition of
    T x_1 F_1^T ... x_N F_N^T restricted to the nonzeros), FP64, returned as an
    N-d array of shape (K_1..K_N)."""
    vals = np.asarray(vals, np.float64)
    K = [np.asarray(f).shape[1] for f in factors]
    G = np.zeros(int(np.prod(K)), np.float64)
    m = vals.shape[0]
    for a in range(0, m, 1 << 15):
        e = np.arange(a, min(a + (1 << 15), m))
        kr = np.ones((len(e), 1))
        for j, f in enumerate(factors):
            rows = np.asarray(f, np.float64)[np.asarray(idx[j])[e]]
            kr = (rows[:, :, None] * kr[:, None, :]).reshape(len(e), -1)   # first index fastest
        G += vals[e] @ kr
    return G.reshape(K, order="F")


def fit_from_norms(norm_t_sq, norm_g_sq):
    if norm_t_sq <= 0:
        return 1.0
    return 1.0 - np.sqrt(max(0.0, norm_t_sq - norm_g_sq)) / np.sqrt(norm_t_sq)


def hooi(idx, vals, dims, factors0, ranks, iters, sweep="gauss_seidel", record=False):
    """Run ``iters`` HOOI invocations from ``factors0``.

    Returns dict(factors, core, fits, sigmas[, history]) where fits[i] is the
    fit after invocation i (core recomputed from the definition each time)."""
    N = len(dims)
    F = [np.asarray(f, np.float64).copy() for f in factors0]
    v = np.asarray(vals, np.float64)
    norm_t_sq = float(v @ v)
    fits, sigmas, history = [], [], []
    for _ in range(iters):
        F_in = [f.copy() for f in F]
        sig_it = []
        for n in range(N):
            src = F if sweep == "gauss_seidel" else F_in
            Z = _ttm.ttm_chain(idx, vals, src, n, dims)
            F[n], s, _ = leading_left_singular_vectors(Z, ranks[n])
            sig_it.append(s)
            if record:
                history.append((n, Z, F[n].copy()))
        G = core(idx, vals, F)
        fits.append(fit_from_norms(norm_t_sq, float(np.sum(G * G))))
        sigmas.append(sig_it)
    out = dict(factors=F, core=core(idx, vals, F), fits=fits, sigmas=sigmas, norm_t_sq=norm_t_sq)
    if record:
        out["history"] = history
    return out


def projector_distance(U, V):
    """||U U^T - V V^T||_F / ||V V^T||_F, free of column signs and rotations."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    # ||UU^T - VV^T||_F^2 = ||U^TU||^2 + ||V^TV||^2 - 2||U^TV||^2 (no L x L matrices)
    a = np.linalg.norm(U.T @ U) ** 2 + np.linalg.norm(V.T @ V) ** 2 - 2 * np.linalg.norm(U.T @ V) ** 2
    return float(np.sqrt(max(a, 0.0)) / np.linalg.norm(V.T @ V))
