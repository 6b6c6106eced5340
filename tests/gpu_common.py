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
