"""Coalescing of the COO element list (oracle; test infrastructure only).

Section 3 represents the tensor as a set E of elements, each a coordinate
vector (l_1, ..., l_N) with a value.  Input lists may repeat a coordinate; the
set view needs each coordinate once, so repeated coordinates are merged by
summing their values (the TTM-chain is linear, so the penultimate matrix is
unchanged by merging; only |E| and ||T|| change).

Canonical order: lexicographic on (l_1, ..., l_N), l_1 most significant.
Duplicates are summed in FP64 in input order, then rounded once to FP32.
"""
from __future__ import annotations

import numpy as np


def coalesce(idx, vals):
    """Return (idx_c: list of N int32 arrays, vals_c: float32 array, norm_sq: float).

    idx: N int arrays of length m (0-based coordinates); vals: m values.
    """
    idx = [np.asarray(i, dtype=np.int64) for i in idx]
    v = np.asarray(vals, dtype=np.float32).astype(np.float64)
    m = v.shape[0]
    if m == 0:
        return [np.zeros(0, np.int32) for _ in idx], np.zeros(0, np.float32), 0.0
    # np.lexsort sorts by the LAST key first; pass keys least significant first.
    order = np.lexsort(tuple(idx[::-1]))  # stable: equal coordinates keep input order
    sidx = [i[order] for i in idx]
    sv = v[order]
    new = np.ones(m, dtype=bool)
    for i in sidx:
        new[1:] &= i[1:] == i[:-1]
    new = ~new
    new[0] = True
    starts = np.flatnonzero(new)
    # Sequential FP64 sums in input order within each run.
    sums = np.empty(starts.shape[0], np.float64)
    ends = np.append(starts[1:], m)
    for k, (a, b) in enumerate(zip(starts, ends)):
        s = 0.0
        for x in sv[a:b]:
            s += float(x)
        sums[k] = s
    vals_c = sums.astype(np.float32)
    idx_c = [i[starts].astype(np.int32) for i in sidx]
    v64 = vals_c.astype(np.float64)
    return idx_c, vals_c, float(np.dot(v64, v64))


def coalesce_fast(idx, vals):
    """Same result as coalesce(), vectorised for large inputs (runs of length
    1 need no summation; longer runs are summed in input order)."""
    idx = [np.asarray(i, dtype=np.int64) for i in idx]
    v = np.asarray(vals, dtype=np.float32).astype(np.float64)
    m = v.shape[0]
    if m == 0:
        return [np.zeros(0, np.int32) for _ in idx], np.zeros(0, np.float32), 0.0
    order = np.lexsort(tuple(idx[::-1]))
    sidx = [i[order] for i in idx]
    sv = v[order]
    same = np.ones(m - 1, dtype=bool)
    for i in sidx:
        same &= i[1:] == i[:-1]
    new = np.ones(m, dtype=bool)
    new[1:] = ~same
    starts = np.flatnonzero(new)
    ends = np.append(starts[1:], m)
    sums = sv[starts].copy()
    multi = np.flatnonzero(ends - starts > 1)
    for k in multi:
        s = 0.0
        for x in sv[starts[k]:ends[k]]:
            s += float(x)
        sums[k] = s
    vals_c = sums.astype(np.float32)
    idx_c = [i[starts].astype(np.int32) for i in sidx]
    v64 = vals_c.astype(np.float64)
    return idx_c, vals_c, float(np.dot(v64, v64))
