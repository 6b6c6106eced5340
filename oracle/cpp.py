"""The oracle's large-input steps in C++17/OpenMP (oracle; test infrastructure only).

Compiled with g++ from three sources into one library:
  ttm_omp.cpp   the TTM-chain (eq. 1, Appendix A; FP64), the same definition as
                ``ttm.py``: ``ttm_chain`` (full Z_(n), timed by the benchmark's
                CPU baseline on the host's cores) and ``RowAccumulator`` (rows of
                chosen slices over elements streamed in batches);
  coo_omp.cpp   coalescing (Section 3) of billions of draws: ``DistinctCounter``
                (merged slice cardinalities of every mode) and ``KeySums`` (merged
                values of chosen coordinates), the same rule as ``coo.py``;
  lite_seq.cpp  Lite (Section 6, its pseudocode figure) with the readings of
                ``lite.py``, for millions of slices and bins: ``lite``.
Pinned against the NumPy oracle and the dense definitions in
tests/test_oracle_ttm.py, tests/test_oracle_lite.py and tests/test_oracle_coo.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("ttm_omp.cpp", "coo_omp.cpp", "lite_seq.cpp")]
_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the sources into liboracle_omp.so (g++, OpenMP)."""
    stale = not os.path.exists(_LIB_PATH) or any(os.path.getmtime(_LIB_PATH) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared"] + _SRCS + ["-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            p, i64 = ctypes.c_void_p, ctypes.c_int64
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_threads.argtypes = []
            lib.oracle_ttm_rows_add.restype = None
            lib.oracle_ttm_rows_add.argtypes = [ctypes.c_int, ctypes.c_int, p, i64, p, p, p, p, i64, p]
            lib.oracle_ttm_chain.restype = None
            lib.oracle_ttm_chain.argtypes = [ctypes.c_int, ctypes.c_int, p, p, i64, p, p, p, p]
            lib.oracle_distinct_new.restype = p
            lib.oracle_distinct_new.argtypes = [ctypes.c_int, p]
            lib.oracle_distinct_add.restype = None
            lib.oracle_distinct_add.argtypes = [p, i64, p]
            lib.oracle_distinct_finish.restype = i64
            lib.oracle_distinct_finish.argtypes = [p, p]
            lib.oracle_distinct_free.restype = None
            lib.oracle_distinct_free.argtypes = [p]
            lib.oracle_keysums_new.restype = p
            lib.oracle_keysums_new.argtypes = [ctypes.c_int, i64, p, i64]
            lib.oracle_keysums_add.restype = None
            lib.oracle_keysums_add.argtypes = [p, i64, p, p]
            lib.oracle_keysums_finish.restype = None
            lib.oracle_keysums_finish.argtypes = [p, p, p]
            lib.oracle_keysums_free.restype = None
            lib.oracle_keysums_free.argtypes = [p]
            lib.oracle_lite.restype = i64
            lib.oracle_lite.argtypes = [i64, p, i64, p, p, p, p, p]
            _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle runs on (OMP_NUM_THREADS, else the cores)."""
    return int(_L().oracle_threads())


def _ptrs(arrays, ctype=ctypes.c_void_p):
    return (ctype * len(arrays))(*[a.ctypes.data for a in arrays])


def ttm_chain(idx, vals, factors, n, dims):
    """Full Z_(n) (dims[n] x Khat_n, FP64) by eq. 1."""
    N = len(dims)
    idx = [np.ascontiguousarray(i, np.int32) for i in idx]
    vals = np.ascontiguousarray(vals, np.float32)
    F = [np.ascontiguousarray(f, np.float64) for f in factors]
    K = np.array([f.shape[1] for f in F], np.int64)
    d = np.array(dims, np.int64)
    khat = int(np.prod([K[j] for j in range(N) if j != n]))
    out = np.empty((int(dims[n]), khat), np.float64)
    _L().oracle_ttm_chain(N, n, d.ctypes.data, K.ctypes.data, vals.shape[0], _ptrs(idx), vals.ctypes.data,
                          _ptrs(F), out.ctypes.data)
    return out


class RowAccumulator:
    """Rows Z_(n)[l, :] of chosen slices, summed over elements fed in batches
    (eq. 1 is a sum over elements, so any split of the element list gives the
    same rows up to the order of FP64 additions)."""

    def __init__(self, factors, n, L_n, slice_ids):
        self.F = [np.ascontiguousarray(f, np.float64) for f in factors]
        self.N = len(self.F)
        self.n = n
        self.K = np.array([f.shape[1] for f in self.F], np.int64)
        self.slice_ids = np.asarray(slice_ids, np.int64)
        self.sel = np.full(int(L_n), -1, np.int32)
        self.sel[self.slice_ids] = np.arange(len(self.slice_ids), dtype=np.int32)
        khat = int(np.prod([self.K[j] for j in range(self.N) if j != n]))
        self.rows = np.zeros((len(self.slice_ids), khat), np.float64)

    def add(self, idx, vals):
        idx = [np.ascontiguousarray(i, np.int32) for i in idx]
        vals = np.ascontiguousarray(vals, np.float32)
        _L().oracle_ttm_rows_add(self.N, self.n, self.K.ctypes.data, vals.shape[0], _ptrs(idx), vals.ctypes.data,
                                 _ptrs(self.F), self.sel.ctypes.data, self.rows.shape[0], self.rows.ctypes.data)


class DistinctCounter:
    """Merged slice cardinalities of every mode of a drawn element list fed in
    batches (repeated coordinates count once, Section 3)."""

    def __init__(self, dims):
        self.dims = tuple(int(d) for d in dims)
        d = np.array(self.dims, np.int64)
        self.h = _L().oracle_distinct_new(len(self.dims), d.ctypes.data)
        if not self.h:
            raise ValueError("coordinates do not pack into the key")

    def add(self, idx):
        idx = [np.ascontiguousarray(i, np.int32) for i in idx]
        _L().oracle_distinct_add(self.h, idx[0].shape[0], _ptrs(idx))

    def finish(self):
        """(number of distinct coordinates, per-mode merged slice sizes)."""
        counts = [np.zeros(L, np.int64) for L in self.dims]
        m = _L().oracle_distinct_finish(self.h, _ptrs(counts))
        _L().oracle_distinct_free(self.h)
        self.h = None
        return int(m), counts


class KeySums:
    """Merged values of chosen (distinct) coordinates: the FP64 sum, in input
    order, of the values of all their draws, rounded once to FP32."""

    def __init__(self, coords, L0):
        self.coords = [np.ascontiguousarray(c, np.int32) for c in coords]
        self.n = self.coords[0].shape[0]
        self.h = _L().oracle_keysums_new(len(self.coords), self.n, _ptrs(self.coords), int(L0))

    def add(self, idx, vals):
        idx = [np.ascontiguousarray(i, np.int32) for i in idx]
        vals = np.ascontiguousarray(vals, np.float32)
        _L().oracle_keysums_add(self.h, vals.shape[0], _ptrs(idx), vals.ctypes.data)

    def finish(self):
        out = np.empty(self.n, np.float32)
        cnt = np.empty(self.n, np.int64)
        _L().oracle_keysums_finish(self.h, out.ctypes.data, cnt.ctypes.data)
        _L().oracle_keysums_free(self.h)
        self.h = None
        return out, cnt


def lite(sizes, P):
    """Lite on per-slice cardinalities (Section 6): the statistics and the
    segments (bin, slice, count, bad) in layout order, as lite.lite gives them."""
    sizes = np.ascontiguousarray(sizes, np.int64)
    L = sizes.shape[0]
    cap = L + int(P)
    seg = [np.empty(cap, np.int64) for _ in range(3)]
    bad = np.empty(cap, np.uint8)
    st = np.empty(7, np.int64)
    S = _L().oracle_lite(L, sizes.ctypes.data, int(P), st.ctypes.data, seg[0].ctypes.data, seg[1].ctypes.data,
                         seg[2].ctypes.data, bad.ctypes.data)
    if S < 0:
        raise AssertionError("stage 2 ran out of bins")
    stats = dict(P=int(P), limit=int(st[0]), m=int(st[1]), L_nonempty=int(st[2]), n_stage1=int(st[3]),
                 E_max=int(st[4]), R_sum=int(S), R_max=int(st[5]), n_bad=int(st[6]))
    return stats, seg[0][:S], seg[1][:S], seg[2][:S], bad[:S]
