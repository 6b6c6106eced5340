"""Seeded synthetic inputs for sparse Tucker workloads.

The sampling code lives in ``gen.c`` (SplitMix64 in counter mode, Zipf by
inverse CDF over a seeded permutation, lognormal by Box-Muller).  This module
only builds that file with gcc and wraps it.  It holds none of the
decomposition's arithmetic; the FP64 checker and the GPU library both consume
the arrays it returns, so they always see identical bytes.

Workload recipes (``make_workload``) mirror the five configurations the
library is measured on; see ``WORKLOADS``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            u64, i64, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
            lib.synth_u01.argtypes = [u64, u64, i64, p]
            lib.synth_normal.argtypes = [u64, u64, i64, p]
            lib.synth_lognormal_f32.argtypes = [u64, u64, i64, p]
            lib.synth_uniform_f32.argtypes = [u64, u64, i64, p]
            lib.synth_perm.argtypes = [u64, u64, i64, p]
            lib.synth_uniform_idx.argtypes = [u64, u64, i64, i64, p]
            lib.synth_zipf_idx.argtypes = [u64, u64, ctypes.c_double, i64, p, i64, p]
            lib.synth_zipf_table.argtypes = [ctypes.c_double, i64, p]
            lib.synth_zipf_guide.argtypes = [p, i64, ctypes.c_int, p]
            lib.synth_zipf_idx_range.argtypes = [u64, u64, p, p, ctypes.c_int, i64, p, i64, i64, p]
            lib.synth_lognormal_f32_range.argtypes = [u64, u64, i64, i64, p]
            for f in (lib.synth_u01, lib.synth_normal, lib.synth_lognormal_f32, lib.synth_uniform_f32,
                      lib.synth_perm, lib.synth_uniform_idx, lib.synth_zipf_idx,
                      lib.synth_zipf_table, lib.synth_zipf_guide, lib.synth_zipf_idx_range,
                      lib.synth_lognormal_f32_range):
                f.restype = None
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# Stream ids inside one seed.
S_IDX = 0          # + mode: coordinate draws of mode n
S_VAL = 100        # values
S_FACTOR = 200     # + mode: initial factor entries
S_PERM = 300       # + mode: Zipf rank -> coordinate permutation
S_CORE = 400       # planted core
S_PLANT = 500      # + mode: planted factors
S_NOISE = 600      # observation noise


def u01(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _L().synth_u01(seed, stream, n, _ptr(out))
    return out


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _L().synth_normal(seed, stream, n, _ptr(out))
    return out


def lognormal_f32(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float32)
    _L().synth_lognormal_f32(seed, stream, n, _ptr(out))
    return out


def uniform_f32(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float32)
    _L().synth_uniform_f32(seed, stream, n, _ptr(out))
    return out


def permutation(seed: int, stream: int, L: int) -> np.ndarray:
    out = np.empty(L, np.int32)
    _L().synth_perm(seed, stream, L, _ptr(out))
    return out


def uniform_idx(seed: int, stream: int, L: int, n: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    _L().synth_uniform_idx(seed, stream, L, n, _ptr(out))
    return out


def zipf_idx_plain(seed: int, stream: int, s: float, L: int, n: int, perm: np.ndarray | None = None) -> np.ndarray:
    """Zipf draws by the plain inverse-CDF binary search over the whole table."""
    if perm is None:
        perm = permutation(seed, S_PERM + stream, L)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    assert perm.shape == (L,)
    out = np.empty(n, np.int32)
    _L().synth_zipf_idx(seed, stream, float(s), L, _ptr(perm), n, _ptr(out))
    return out


GUIDE_LOG2 = 20   # buckets of the guided Zipf search


class ZipfSampler:
    """Zipf(s) draws over a permuted [0, L) in any range of the counter: the
    inverse-CDF search narrowed by a guide table (same draws as
    zipf_idx_plain, bit for bit)."""

    def __init__(self, seed: int, stream: int, s: float, L: int, perm: np.ndarray | None = None):
        self.seed, self.stream, self.L = int(seed), int(stream), int(L)
        if perm is None:
            perm = permutation(seed, S_PERM + stream, L)
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)
        assert self.perm.shape == (L,)
        self.table = np.empty(L, np.float64)
        _L().synth_zipf_table(float(s), L, _ptr(self.table))
        self.guide = np.empty((1 << GUIDE_LOG2) + 1, np.int64)
        _L().synth_zipf_guide(_ptr(self.table), L, GUIDE_LOG2, _ptr(self.guide))

    def draw(self, start: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
        if out is None:
            out = np.empty(n, np.int32)
        assert out.dtype == np.int32 and out.flags["C_CONTIGUOUS"] and out.shape[0] >= n
        _L().synth_zipf_idx_range(self.seed, self.stream, _ptr(self.table), _ptr(self.guide), GUIDE_LOG2, self.L,
                                  _ptr(self.perm), int(start), int(n), _ptr(out))
        return out[:n]


def zipf_idx(seed: int, stream: int, s: float, L: int, n: int, perm: np.ndarray | None = None) -> np.ndarray:
    return ZipfSampler(seed, stream, s, L, perm).draw(0, n)


def lognormal_f32_range(seed: int, stream: int, start: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
    if out is None:
        out = np.empty(n, np.float32)
    assert out.dtype == np.float32 and out.flags["C_CONTIGUOUS"] and out.shape[0] >= n
    _L().synth_lognormal_f32_range(seed, stream, int(start), int(n), _ptr(out))
    return out[:n]


def gaussian_factors(seed: int, dims, ranks):
    """Seeded Gaussian L_n x K_n matrices (FP64, row-major), one stream per mode."""
    return [normal(seed, S_FACTOR + n, int(L) * int(K)).reshape(int(L), int(K)) for n, (L, K) in
            enumerate(zip(dims, ranks))]


def orthonormal_init(seed: int, dims, ranks):
    """Initial factors: seeded Gaussian then Householder QR (numpy), columns
    signed so that diag(R) > 0.  Harness-side initialisation, fed to both the
    checker and the library."""
    out = []
    for A in gaussian_factors(seed, dims, ranks):
        Q, R = np.linalg.qr(A)
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        out.append(np.ascontiguousarray(Q * d))
    return out


# ----------------------------------------------------------------------------------------------
# Workload recipes.  Tensor seed 1804 + c, factor seed 9494 + c (c = workload number),
# planted-model seed 4949.
# ----------------------------------------------------------------------------------------------

WORKLOADS = {
    "c1": dict(dims=(200, 150, 100), nnz=20_000, dist="uniform", values="uniform",
               ranks=(5, 5, 5), iters=3, number=1),
    "c2": dict(dims=(1_000_000, 500_000, 200_000), nnz=100_000_000, dist="zipf", zipf=(1.1, 1.1, 1.1),
               values="lognormal", ranks=(10, 10, 10), iters=5, number=2),
    "c3": dict(dims=(2_000_000, 1_000_000, 100_000, 5_000), nnz=500_000_000, dist="zipf",
               zipf=(0.9, 1.1, 1.3, 0.7), values="lognormal", ranks=(10, 10, 10, 10), iters=3, number=3),
    "c4": dict(dims=(500_000, 500_000, 50_000), nnz=200_000_000, dist="zipf", zipf=(1.0, 1.0, 1.0),
               values="planted", ranks=(16, 16, 16), number=4),
    "c5": dict(dims=(4_000_000, 4_000_000, 2_000_000), nnz=4_000_000_000, dist="zipf",
               zipf=(0.8, 1.2, 1.5), values="lognormal", ranks=(10, 10, 10), iters=1, number=5),
}


def coordinates(seed: int, dims, nnz: int, dist: str, zipf=None):
    """N int32 coordinate arrays (0-based) of nnz draws."""
    out = []
    for n, L in enumerate(dims):
        if dist == "uniform":
            out.append(uniform_idx(seed, S_IDX + n, int(L), nnz))
        elif dist == "zipf":
            out.append(zipf_idx(seed, S_IDX + n, float(zipf[n]), int(L), nnz))
        else:
            raise ValueError(dist)
    return out


def values(seed: int, nnz: int, kind: str) -> np.ndarray:
    if kind == "uniform":
        return uniform_f32(seed, S_VAL, nnz)
    if kind == "lognormal":
        return lognormal_f32(seed, S_VAL, nnz)
    raise ValueError(kind)


def make_tensor(dims, nnz, dist="zipf", zipf=None, values_kind="lognormal", seed=1804):
    """(idx list of N int32 arrays, float32 values) for a synthetic sparse tensor."""
    idx = coordinates(seed, dims, nnz, dist, zipf)
    return idx, values(seed, nnz, values_kind)


def make_workload(name: str, scale: float = 1.0, share: int = 1):
    """Coordinates, values, initial factors and ranks of a named workload.

    ``scale`` < 1 shrinks dims and nnz by that factor (same distributions),
    used for parity cases the checker finishes in seconds.  ``share`` > 1 keeps
    the dims and takes the first nnz/share draws: one GPU's part of the
    workload spread over ``share`` GPUs (the draws are counter-based, so this
    is exactly the first contiguous shard)."""
    w = dict(WORKLOADS[name])
    c = w["number"]
    dims = tuple(max(2, int(round(L * scale))) for L in w["dims"])
    nnz = max(1, int(round(w["nnz"] * scale)) // max(1, int(share)))
    if w["values"] == "planted":
        raise ValueError("use make_completion for the planted-model workload")
    idx, vals = make_tensor(dims, nnz, w["dist"], w.get("zipf"), w["values"], seed=1804 + c)
    ranks = tuple(min(k, L) for k, L in zip(w["ranks"], dims))
    F0 = orthonormal_init(9494 + c, dims, ranks)
    return dict(dims=dims, idx=idx, vals=vals, ranks=ranks, F0=F0, iters=w.get("iters", 1))


class WorkloadStream:
    """A named Zipf workload drawn in consecutive chunks of the counter range
    (the same draws as make_workload, chunk by chunk), for inputs too large to
    hold at once.  chunk(start, n) fills caller buffers (idx: N int32 arrays,
    vals: float32) with draws start .. start+n-1."""

    def __init__(self, name: str, scale: float = 1.0, share: int = 1):
        w = dict(WORKLOADS[name])
        if w["dist"] != "zipf" or w["values"] != "lognormal":
            raise ValueError("streamed workloads are the Zipf / lognormal ones")
        c = w["number"]
        self.name = name
        self.seed = 1804 + c
        self.dims = tuple(max(2, int(round(L * scale))) for L in w["dims"])
        self.nnz = max(1, int(round(w["nnz"] * scale)) // max(1, int(share)))
        self.ranks = tuple(min(k, L) for k, L in zip(w["ranks"], self.dims))
        self.zipf = w["zipf"]
        self.iters = w.get("iters", 1)
        self.samplers = [ZipfSampler(self.seed, S_IDX + n, float(self.zipf[n]), int(L))
                         for n, L in enumerate(self.dims)]
        self.factor_seed = 9494 + c

    def chunk(self, start: int, n: int, idx=None, vals=None):
        N = len(self.dims)
        if idx is None:
            idx = [np.empty(n, np.int32) for _ in range(N)]
        if vals is None:
            vals = np.empty(n, np.float32)
        for j in range(N):
            self.samplers[j].draw(start, n, idx[j])
        lognormal_f32_range(self.seed, S_VAL, start, n, vals)
        return [a[:n] for a in idx], vals[:n]

    def initial_factors(self):
        return orthonormal_init(self.factor_seed, self.dims, self.ranks)


def make_completion(dims, n_obs, ranks, zipf=(1.0, 1.0, 1.0), noise=0.01, seed=4949):
    """Observation coordinates of a completion problem and a planted model
    (core ~ N(0,1), factors ~ N(0, 1/K_n)) with N(0, noise^2) draws per
    observation.  The targets are the planted model's values plus the noise;
    evaluating the model is the caller's (this module does no Tucker
    arithmetic)."""
    N = len(dims)
    idx = [zipf_idx(seed, S_IDX + n, float(zipf[n]), int(dims[n]), n_obs) for n in range(N)]
    K = list(ranks)
    G = normal(seed, S_CORE, int(np.prod(K))).reshape(K, order="F")
    F = [normal(seed, S_PLANT + n, int(dims[n]) * K[n]).reshape(int(dims[n]), K[n]) / np.sqrt(K[n])
         for n in range(N)]
    return dict(dims=tuple(dims), idx=idx, ranks=tuple(ranks), G_true=G, F_true=F,
                noise=noise * normal(seed, S_NOISE, n_obs))
