"""Helpers shared by the GPU parity tests (input construction and comparisons)."""
import numpy as np

import synth
from oracle import coo, hooi, lite, ttm


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def zipf_tensor(dims, nnz, s=1.1, seed=11, values="lognormal"):
    z = s if isinstance(s, (tuple, list)) else tuple([s] * len(dims))
    idx, vals = synth.make_tensor(dims, nnz, "zipf", z, values, seed=seed)
    return idx, vals


def uniform_tensor(dims, nnz, seed=3):
    return synth.make_tensor(dims, nnz, "uniform", None, "uniform", seed=seed)


def oracle_partition(idx_c, dims, n, P):
    return lite.partition_mode(idx_c[n], dims[n], P)


def oracle_Y(idx_c, vals_c, F, n, dims):
    Y = ttm.ttm_chain(idx_c, vals_c, F, n, dims)
    rows = ttm.nonempty_slices(idx_c[n], dims[n])
    return Y[rows], rows


U32 = 2.0 ** -24   # FP32 unit roundoff


def factor_tolerance(sv, K, tol=1e-5):
    """Allowed projector distance of a GPU factor from the oracle's.

    Where the oracle's spectrum separates the leading K-subspace
    (sigma_K / sigma_{K+1} - 1 >= 1e-3) the bar is tol.  Below that, the
    sin-theta theorem bounds the subspace error of an eigensolve of a Gram
    matrix with FP32 perturbation ||E|| <= c u sigma_1^2 by
    sqrt(2) c u sigma_1^2 / (sigma_K^2 - sigma_{K+1}^2); c = 4 covers the FP32
    rounding of Y and of the Gram's accumulation."""
    if len(sv) <= K or sv[K] == 0.0 or sv[K - 1] / sv[K] - 1.0 >= 1e-3:
        return tol, 1.0
    cond = sv[0] ** 2 / max(sv[K - 1] ** 2 - sv[K] ** 2, 1e-300)
    return max(tol, np.sqrt(2.0) * 4.0 * U32 * cond), cond


def factor_tolerance_y(sv, K, tol=1e-5):
    """Allowed projector distance for an SVD step that never squares Y (the
    matrix-free route: products with Y in FP64 from its FP32 entries).  The
    perturbation is Y's own rounding, ||E|| <= c u sigma_1, and Wedin's
    sin-theta theorem bounds the subspace error by
    sqrt(2) c u sigma_1 / (sigma_K - sigma_{K+1}); c = 4 as above."""
    if len(sv) <= K or sv[K] == 0.0:
        return tol
    return max(tol, np.sqrt(2.0) * 4.0 * U32 * sv[0] / max(sv[K - 1] - sv[K], 1e-300))


def fit_noise(fit):
    """Rounding noise of the fit 1 - sqrt(||T||^2 - ||G||^2)/||T|| when
    ||G||^2 carries a relative FP32 error of c u (c = 4, from Y and the core's
    accumulation): delta fit <= c u / (2 (1 - fit)) for ||G|| <= ||T||, and a
    difference of two such values at most twice that.  Fits that should not
    decrease (Gauss-Seidel HOOI) are allowed to drop by this much."""
    return max(1e-6, 4.0 * U32 / max(1.0 - fit, 1e-12))


def completion_targets(d):
    """Targets of a synth.make_completion problem: the planted model's values
    (oracle) plus the generator's noise, rounded to FP32."""
    from oracle import completion
    return (completion.model_values(d["G_true"], d["F_true"], d["idx"]) + d["noise"]).astype(np.float32)
