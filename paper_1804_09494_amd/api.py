"""Python binding of the tucker_hip C ABI: argument marshalling only.

Every computation runs in libtucker_hip.so.  Arrays may be NumPy arrays
(host memory) or torch tensors (CUDA tensors are passed as device pointers,
CPU tensors as host pointers); torch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (TK_MEM_DEVICE, TK_MEM_HOST, TuckerError, c_f64, c_i32, c_i64, c_int, c_void_p, tk_options,
                   tk_part_stats)

try:
    import torch
except Exception:  # torch is optional for host-memory use
    torch = None


def _is_torch(x):
    return torch is not None and isinstance(x, torch.Tensor)


def _mem_of(x):
    if _is_torch(x):
        return TK_MEM_DEVICE if x.is_cuda else TK_MEM_HOST
    return TK_MEM_HOST


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return c_void_p(x.data_ptr())
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return x.ctypes.data_as(c_void_p)


def _check_dtype(x, np_dtype, name):
    if _is_torch(x):
        want = {np.int32: torch.int32, np.float32: torch.float32, np.float64: torch.float64, np.int64: torch.int64,
                np.uint8: torch.uint8}[np_dtype]
        if x.dtype != want:
            raise TypeError(f"{name}: expected {want}, got {x.dtype}")
    elif np.asarray(x).dtype != np_dtype:
        raise TypeError(f"{name}: expected {np.dtype(np_dtype)}, got {np.asarray(x).dtype}")


def _current_stream(device):
    if torch is not None and torch.cuda.is_available():
        return c_void_p(torch.cuda.current_stream(device).cuda_stream)
    return c_void_p(None)


class TuckerContext:
    """One library context on one GPU (tk_create / tk_destroy)."""

    def __init__(self, device: int = 0, stream=None, allocator=None, **options):
        """allocator: None (the library's hipMalloc / hipFree) or "torch" (torch's
        caching allocator backs every device allocation of the context, on the
        context's stream)."""
        self._L = _lib.load()
        h = c_void_p()
        if stream is None:
            stream = _current_stream(device)
        elif _is_torch_stream(stream):
            stream = c_void_p(stream.cuda_stream)
        self._opt = None
        self._alloc = None
        if allocator == "torch":
            self._alloc = _torch_allocator(device, stream.value or 0)
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        self._check(self._L.tk_create(device, stream, ctypes.byref(self._alloc) if self._alloc else None,
                                      ctypes.byref(h)), None)
        self._h = h
        self.device = device
        self.N = 0
        self.dims = ()
        self.ranks = ()
        if options:
            self.set_options(**options)

    # -- plumbing --
    def _check(self, status, h="self"):
        if status != _lib.TK_OK:
            msg = self._L.tk_last_error(self._h if h == "self" else None)
            raise TuckerError(status, (msg or b"").decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.tk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        s = c_void_p(stream.cuda_stream) if _is_torch_stream(stream) else c_void_p(stream)
        self._check(self._L.tk_set_stream(self._h, s))

    def options(self) -> tk_options:
        """A copy of the options in effect (the defaults until set_options)."""
        o = tk_options()
        if self._opt is None:
            self._L.tk_default_options(ctypes.byref(o))
        else:
            ctypes.memmove(ctypes.byref(o), ctypes.byref(self._opt), ctypes.sizeof(o))
        return o

    def set_options(self, **kw):
        """Change the named options; the others keep their current values."""
        o = self.options()
        prec = kw.pop("prec", None)
        if prec is not None:
            o.prec = {"fp32": _lib.TK_FP32, "bf16": _lib.TK_BF16}.get(prec, prec)
        part = kw.pop("partition", None)
        if part is not None:
            o.partition = {"lite": _lib.TK_PART_LITE, "coarse": _lib.TK_PART_COARSE}.get(part, part)
        kern = kw.pop("ttm_kernel", None)
        if kern is not None:
            o.ttm_kernel = {"auto": _lib.TK_TTM_AUTO, "vector": _lib.TK_TTM_VECTOR,
                            "atomic": _lib.TK_TTM_ATOMIC, "fiber": _lib.TK_TTM_FIBER}.get(kern, kern)
        eig = kw.pop("eig_method", None)
        if eig is not None:
            o.eig_method = {"auto": _lib.TK_EIG_AUTO, "gram": _lib.TK_EIG_GRAM,
                            "matfree": _lib.TK_EIG_MATFREE}.get(eig, eig)
        sweep = kw.pop("sweep", None)
        if sweep is not None:
            o.sweep = {"gauss_seidel": _lib.TK_SWEEP_GAUSS_SEIDEL, "jacobi": _lib.TK_SWEEP_JACOBI}.get(sweep, sweep)
        for k, v in kw.items():
            setattr(o, k, v)
        self._check(self._L.tk_set_options(self._h, ctypes.byref(o)))
        self._opt = o

    # -- tensor --
    def load_coo(self, idx, vals, dims, assume_unique=False):
        N = len(dims)
        if len(idx) != N:
            raise ValueError("need one coordinate array per mode")
        mem, nnz = self._check_chunk(idx, vals)
        d = (c_i64 * N)(*[int(x) for x in dims])
        ptrs = (c_void_p * N)(*[_ptr(a) for a in idx])
        flags = _lib.TK_ASSUME_UNIQUE if assume_unique else 0
        self._check(self._L.tk_load_coo(self._h, N, d, nnz, ptrs, _ptr(vals), mem, flags))
        self.N, self.dims = N, tuple(int(x) for x in dims)

    def _check_chunk(self, idx, vals):
        mem = _mem_of(vals)
        nnz = int(vals.shape[0])
        for i, a in enumerate(idx):
            _check_dtype(a, np.int32, f"idx[{i}]")
            if _mem_of(a) != mem or int(a.shape[0]) != nnz:
                raise ValueError("coordinate arrays must match vals in length and memory kind")
        _check_dtype(vals, np.float32, "vals")
        return mem, nnz

    def load_begin(self, dims, nnz, assume_unique=False):
        """Streamed load (tk_load_coo_begin): announce dims and the total
        element count, then load_append the elements in pieces, then load_end."""
        N = len(dims)
        d = (c_i64 * N)(*[int(x) for x in dims])
        flags = _lib.TK_ASSUME_UNIQUE if assume_unique else 0
        self._check(self._L.tk_load_coo_begin(self._h, N, d, int(nnz), flags))
        self._pending = (N, tuple(int(x) for x in dims))

    def load_append(self, idx, vals):
        mem, count = self._check_chunk(idx, vals)
        ptrs = (c_void_p * len(idx))(*[_ptr(a) for a in idx])
        self._check(self._L.tk_load_coo_append(self._h, count, ptrs, _ptr(vals), mem))

    def load_end(self):
        self._check(self._L.tk_load_coo_end(self._h))
        self.N, self.dims = self._pending

    def tensor_info(self):
        m, nsq = c_i64(), c_f64()
        self._check(self._L.tk_get_tensor_info(self._h, ctypes.byref(m), ctypes.byref(nsq)))
        return m.value, nsq.value

    def get_coo(self):
        m, _ = self.tensor_info()
        idx = [np.empty(m, np.int32) for _ in range(self.N)]
        vals = np.empty(m, np.float32)
        ptrs = (c_void_p * self.N)(*[_ptr(a) for a in idx])
        self._check(self._L.tk_get_coo(self._h, ptrs, _ptr(vals), TK_MEM_HOST))
        return idx, vals

    # -- ranks and partition --
    def set_ranks(self, ranks):
        K = (c_i32 * self.N)(*[int(k) for k in ranks])
        self._check(self._L.tk_set_ranks(self._h, K))
        self.ranks = tuple(int(k) for k in ranks)

    def set_slice_order(self, n, perm):
        """The random slice order of mode n for the CoarseG partition."""
        _check_dtype(perm, np.int32, "perm")
        self._check(self._L.tk_set_slice_order(self._h, n, _ptr(perm), _mem_of(perm)))

    def partition_stats(self, n):
        s = tk_part_stats()
        self._check(self._L.tk_get_partition_stats(self._h, n, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in tk_part_stats._fields_}

    def partition(self, n, elem_order=True):
        st = self.partition_stats(n)
        P, S, m = st["P"], st["R_sum"], st["m"]
        out = dict(bin_ptr=np.empty(P + 1, np.int64), seg_bin=np.empty(S, np.int32),
                   seg_slice=np.empty(S, np.int32), seg_begin=np.empty(S + 1, np.int64),
                   seg_bad=np.empty(S, np.uint8))
        eo = np.empty(m, np.int64) if elem_order else None
        self._check(self._L.tk_get_partition(self._h, n, _ptr(out["bin_ptr"]), _ptr(eo), _ptr(out["seg_bin"]),
                                             _ptr(out["seg_slice"]), _ptr(out["seg_begin"]), _ptr(out["seg_bad"]),
                                             TK_MEM_HOST))
        if elem_order:
            out["elem_order"] = eo
        out["stats"] = st
        return out

    # -- factors --
    def set_factor(self, n, F):
        _check_dtype(F, np.float64, "F")
        if tuple(F.shape) != (self.dims[n], self.ranks[n]):
            raise ValueError(f"factor {n} must be {self.dims[n]} x {self.ranks[n]}")
        self._check(self._L.tk_set_factor(self._h, n, _ptr(F), _mem_of(F)))

    def get_factor(self, n, out=None):
        if out is None:
            out = np.empty((self.dims[n], self.ranks[n]), np.float64)
        self._check(self._L.tk_get_factor(self._h, n, _ptr(out), _mem_of(out)))
        return out

    # -- hot path --
    def ttm_shape(self, n):
        R, kh = c_i64(), c_i64()
        self._check(self._L.tk_ttm_shape(self._h, n, ctypes.byref(R), ctypes.byref(kh)))
        return R.value, kh.value

    def ttm_chain(self, n, Y=None, row_slice=None, device=None):
        """Y_(n) (R_n x Khat_n FP32) and its row slice ids.  With device=True
        (or torch output tensors on the GPU) the result stays in device memory."""
        R, kh = self.ttm_shape(n)
        if Y is None:
            if device:
                Y = torch.empty((R, kh), dtype=torch.float32, device=f"cuda:{self.device}")
                row_slice = torch.empty(R, dtype=torch.int32, device=f"cuda:{self.device}")
            else:
                Y = np.empty((R, kh), np.float32)
                row_slice = np.empty(R, np.int32)
        mem = _mem_of(Y)
        self._check(self._L.tk_ttm_chain(self._h, n, _ptr(Y), _ptr(row_slice), mem))
        return Y, row_slice

    def ttm_chain_noalloc(self, n, Y, row_slice=None):
        """tk_ttm_chain_noalloc into caller-allocated device tensors (Y: R_n x
        Khat_n float32, row_slice: R_n int32 or None); nothing is allocated."""
        _check_dtype(Y, np.float32, "Y")
        if row_slice is not None:
            _check_dtype(row_slice, np.int32, "row_slice")
        self._check(self._L.tk_ttm_chain_noalloc(self._h, n, _ptr(Y), _ptr(row_slice)))
        return Y, row_slice

    def hooi_iterate(self, iters):
        fits = np.zeros(max(iters, 1), np.float64)
        self._check(self._L.tk_hooi_iterate(self._h, iters, _ptr(fits)))
        return fits[:iters].tolist()

    def init_hosvd(self, sketches):
        """tk_init_hosvd: factors from the Kronecker-sketched HOSVD; sketches[j]
        is L_j x K_j float64 (all host arrays or all device tensors).
        Returns the fit of the initial decomposition."""
        if len(sketches) != self.N:
            raise ValueError(f"need {self.N} sketch matrices")
        mem = _mem_of(sketches[0])
        for j, S in enumerate(sketches):
            _check_dtype(S, np.float64, "sketch")
            if tuple(S.shape) != (self.dims[j], self.ranks[j]) or _mem_of(S) != mem:
                raise ValueError(f"sketch {j} must be {self.dims[j]} x {self.ranks[j]}, all on one side")
        ptrs = (c_void_p * self.N)(*[_ptr(S) for S in sketches])
        fit = c_f64()
        self._check(self._L.tk_init_hosvd(self._h, ptrs, mem, ctypes.byref(fit)))
        return fit.value

    def core(self):
        out = np.empty(int(np.prod(self.ranks)), np.float64)
        fit = c_f64()
        self._check(self._L.tk_core(self._h, _ptr(out), ctypes.byref(fit), TK_MEM_HOST))
        return out.reshape(self.ranks, order="F"), fit.value

    def timings(self):
        cap = c_int(64)
        ms = (c_f64 * 64)()
        names = (ctypes.c_char_p * 64)()
        self._check(self._L.tk_get_timings(self._h, ms, names, ctypes.byref(cap)))
        return {names[i].decode(): ms[i] for i in range(cap.value)}

    def counters(self):
        cap = c_int(16)
        vals = (c_i64 * 16)()
        names = (ctypes.c_char_p * 16)()
        self._check(self._L.tk_get_counters(self._h, vals, names, ctypes.byref(cap)))
        return {names[i].decode(): vals[i] for i in range(cap.value)}

    # -- differentiation form --
    def load_obs(self, idx, dims, ranks):
        N = len(dims)
        n_obs = int(idx[0].shape[0])
        mem = _mem_of(idx[0])
        for i, a in enumerate(idx):
            _check_dtype(a, np.int32, f"idx[{i}]")
        d = (c_i64 * N)(*[int(x) for x in dims])
        K = (c_i32 * N)(*[int(k) for k in ranks])
        ptrs = (c_void_p * N)(*[_ptr(a) for a in idx])
        self._check(self._L.tk_load_obs(self._h, N, d, K, n_obs, ptrs, mem))
        self.obs_dims, self.obs_ranks, self.n_obs = tuple(dims), tuple(ranks), n_obs

    def tucker_eval(self, core, F, out=None):
        mem = _mem_of(core)
        if out is None:
            if mem == TK_MEM_DEVICE:
                out = torch.empty(self.n_obs, dtype=torch.float32, device=core.device)
            else:
                out = np.empty(self.n_obs, np.float32)
        Fp = (c_void_p * len(F))(*[_ptr(f) for f in F])
        self._check(self._L.tk_tucker_eval(self._h, _ptr(core), Fp, _ptr(out), mem))
        return out

    def tucker_adjoint(self, g, core, F):
        mem = _mem_of(core)
        if mem == TK_MEM_DEVICE:
            dcore = torch.empty_like(core)
            dF = [torch.empty_like(f) for f in F]
        else:
            dcore = np.empty_like(core)
            dF = [np.empty_like(f) for f in F]
        Fp = (c_void_p * len(F))(*[_ptr(f) for f in F])
        dFp = (c_void_p * len(F))(*[_ptr(f) for f in dF])
        self._check(self._L.tk_tucker_adjoint(self._h, _ptr(g), _ptr(core), Fp, _ptr(dcore), dFp, mem))
        return dcore, dF


def _torch_allocator(device, stream_handle):
    """tk_allocator whose hooks call torch's caching allocator (the callbacks
    are kept alive by the returned structure's owner)."""
    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream_handle)
        except Exception:   # out of memory: the library reports TK_ERR_OOM
            return None

    def free(ptr, nbytes, user):
        torch.cuda.caching_allocator_delete(ptr)

    a = _lib.tk_allocator(_lib.TK_ALLOC_FN(alloc), _lib.TK_FREE_FN(free), None)
    a._keep = (alloc, free)
    return a


def _is_torch_stream(s):
    return torch is not None and isinstance(s, torch.cuda.Stream)


if torch is not None:
    class TuckerEval(torch.autograd.Function):
        """model = TuckerEval.apply(ctx, core, F_1, ..., F_N): Tucker model values at
        the observations loaded into ``ctx`` (tk_tucker_eval); the backward pass
        calls the hand-written adjoint (tk_tucker_adjoint).  All tensors are FP32
        and contiguous; core is stored first index fastest (flattened)."""

        @staticmethod
        def forward(fctx, tctx, core, *F):
            fctx.tctx = tctx
            fctx.save_for_backward(core, *F)
            return tctx.tucker_eval(core.contiguous(), [f.contiguous() for f in F])

        @staticmethod
        def backward(fctx, g):
            core, *F = fctx.saved_tensors
            dcore, dF = fctx.tctx.tucker_adjoint(g.contiguous(), core.contiguous(), [f.contiguous() for f in F])
            return (None, dcore, *dF)
