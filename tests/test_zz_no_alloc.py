"""The allocation-free TTM-chain (tk_ttm_chain_noalloc) against tk_ttm_chain.

Both run the same kernels, so their outputs must agree bit for bit.  Two
calls in a row share the library's static scratch array: first a larger
tensor (many split slices), then a smaller one on a second context.  The
outputs are preallocated torch tensors, so nothing is allocated around the
calls."""
import numpy as np
import pytest

import synth
from tests.gpu_common import zipf_tensor

pytestmark = pytest.mark.gpu


def _ctx(tk, idx, vals, dims, ranks, wg):
    import torch
    ctx = tk.TuckerContext(0, wg_nnz_target=wg)
    ctx.load_coo([torch.from_numpy(np.ascontiguousarray(i)).cuda() for i in idx],
                 torch.from_numpy(np.ascontiguousarray(vals)).cuda(), dims)
    ctx.set_ranks(ranks)
    F = [synth.normal(61, 200 + n, d * k).reshape(d, k) for n, (d, k) in enumerate(zip(dims, ranks))]
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    return ctx


def _compare(ctx, N):
    import torch
    for n in range(N):
        R, kh = ctx.ttm_shape(n)
        Y = torch.full((R, kh), float("nan"), dtype=torch.float32, device="cuda")
        rows = torch.full((R,), -1, dtype=torch.int32, device="cuda")
        Yr = torch.empty((R, kh), dtype=torch.float32, device="cuda")
        rr = torch.empty((R,), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        ctx.ttm_chain_noalloc(n, Y, rows)
        ctx.ttm_chain(n, Yr, rr)
        torch.cuda.synchronize()
        st = ctx.partition_stats(n)
        print(f"  mode {n}: R={R} Khat={kh} split slices={st['n_bad']}", flush=True)
        assert torch.equal(rows, rr)
        assert torch.equal(Y, Yr)


def test_noalloc_matches_ttm_chain_two_calls(tk):
    # first call: 3-mode matrix-core kernel, small bins so many slices are split
    idx, vals = zipf_tensor((20_000, 8_000, 3_000), 400_000, s=1.3, seed=71)
    dims = tuple(int(i.max()) + 1 for i in idx)
    print("call 1", dims, len(vals), flush=True)
    a = _ctx(tk, idx, vals, dims, (10, 10, 10), 256)
    _compare(a, 3)
    # second call, smaller input on another context: four modes (the four-mode
    # matrix-core kernel and, for rank 20, the vector-ALU one)
    idx, vals = zipf_tensor((300, 200, 100, 40), 20_000, s=1.0, seed=72)
    dims = tuple(int(i.max()) + 1 for i in idx)
    print("call 2", dims, len(vals), flush=True)
    b = _ctx(tk, idx, vals, dims, (20, 6, 5, 4), 512)
    _compare(b, 4)


def test_noalloc_rejects_oversize_scratch(tk):
    import torch
    # one slice of 400,000 elements over bins of 64: ~6,250 partial rows of
    # Khat = 6,000 floats, far above the scratch array
    n_giant = 400_000
    j = np.arange(n_giant, dtype=np.int64)
    idx = [np.zeros(n_giant, np.int32), (j % 1999).astype(np.int32), ((j * 7) % 997).astype(np.int32),
           ((j * 13) % 101).astype(np.int32)]
    vals = np.ones(n_giant, np.float32)
    dims = (4, 1999, 997, 101)
    ctx = _ctx(tk, idx, vals, dims, (2, 20, 20, 15), 64)
    R, kh = ctx.ttm_shape(0)
    st = ctx.partition_stats(0)
    assert st["n_bad"] >= 1 and kh == 6000
    Y = torch.empty((R, kh), dtype=torch.float32, device="cuda")
    with pytest.raises(tk.TuckerError, match="UNSUPPORTED"):
        ctx.ttm_chain_noalloc(0, Y)
    # a host buffer is refused before anything runs
    with pytest.raises(tk.TuckerError, match="INVALID_ARG"):
        ctx.ttm_chain_noalloc(1, np.empty(ctx.ttm_shape(1), np.float32))
