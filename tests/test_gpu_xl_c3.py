"""Parity of the precision form at full size: 4-mode 2,000,000 x 1,000,000 x
100,000 x 5,000, 5e8 draws (Zipf 0.9 / 1.1 / 1.3 / 0.7), lognormal values,
ranks 10 (Y_(n) has 1,000 columns), streamed into the library in chunks.

The oracle cannot form Y_(n) here (2e6 x 1000 in FP64), so it computes, from
the draws and with its C++/OpenMP FP64 code, the rows of Y_(n) for seeded
slices of every mode: the ten heaviest Zipf ranks, the next twenty (which
Lite splits across bins), and thirty random ids.  The library's TTM-chain is
held to 1e-5 in FP32 and to 1e-2 with BF16 Kronecker tiles on those rows;
HOOI is checked by properties (orthonormal factors; a run of BF16
invocations closed by the refining FP32 one ends at the FP32 run's fit to
1e-5)."""
import numpy as np
import pytest

import synth
from oracle import cpp
from tests.gpu_common import rel_fro

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

CHUNK = 1 << 26


@pytest.fixture(scope="module")
def c3(tk):
    import time
    import torch
    stream = synth.WorkloadStream("c3")
    dims, nnz = stream.dims, stream.nnz
    N = len(dims)
    F0 = stream.initial_factors()
    rng = np.random.default_rng(33)
    picks = []
    for n in range(N):
        heavy = stream.samplers[n].perm[:30]                  # Zipf ranks 1 .. 30
        picks.append(np.unique(np.concatenate([heavy, rng.choice(dims[n], 30, replace=False)])))
    accs = [cpp.RowAccumulator(F0, n, dims[n], picks[n]) for n in range(N)]
    ctx = tk.TuckerContext(0, keep_elem_order=0)
    bufs = ([torch.empty(CHUNK, dtype=torch.int32, pin_memory=True).numpy() for _ in range(N)],
            torch.empty(CHUNK, dtype=torch.float32, pin_memory=True).numpy())
    t0 = time.time()
    ctx.load_begin(dims, nnz)
    for a in range(0, nnz, CHUNK):
        n_ = min(CHUNK, nnz - a)
        idx, vals = stream.chunk(a, n_, *bufs)
        ctx.load_append(idx, vals)
        for acc in accs:
            acc.add(idx, vals)
    ctx.load_end()
    print(f"c3 loaded, oracle rows done: {time.time() - t0:.0f}s", flush=True)
    ctx.set_ranks(stream.ranks)
    print(f"partition and layout built, {time.time() - t0:.0f}s", flush=True)
    return dict(stream=stream, ctx=ctx, F0=F0, picks=picks, accs=accs)


def _sampled_rows(ctx, n, pick):
    import torch
    Y, rows = ctx.ttm_chain(n, device=True)
    rows_h = rows.cpu().numpy()
    present = np.isin(pick, rows_h)
    at = torch.from_numpy(np.searchsorted(rows_h, pick[present])).cuda()
    return Y.index_select(0, at).double().cpu().numpy(), present


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c3_ttm_sampled_rows(c3, prec):
    ctx = c3["ctx"]
    ctx.set_options(prec=prec)
    for n, F in enumerate(c3["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    for n in range(4):
        Yg, present = _sampled_rows(ctx, n, c3["picks"][n])
        Yo = c3["accs"][n].rows
        assert np.all(np.linalg.norm(Yo[~present], axis=1) == 0.0)
        err = rel_fro(Yg, Yo[present])
        print(f"{prec} mode {n}: {present.sum()} sampled rows, rel err {err:.2e}", flush=True)
        if prec == "fp32":
            assert err <= 1e-5
        else:
            assert 1e-5 < err <= 1e-2
    ctx.set_options(prec="fp32")


def test_c3_hooi_fp32_and_bf16_runs(c3):
    ctx = c3["ctx"]

    def run(prec, iters):
        ctx.set_options(prec=prec, refine=1)
        for n, F in enumerate(c3["F0"]):
            ctx.set_factor(n, np.ascontiguousarray(F))
        fits = ctx.hooi_iterate(iters)
        return fits, ctx.timings()

    fits, tm = run("fp32", 3)
    for n in range(4):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(10), atol=1e-12)
    bf, tmb = run("bf16", 3)
    print("c3 fits fp32", fits, "bf16 then refined", bf, flush=True)
    print("c3 ttm ms fp32", [round(tm[f"ttm_kernel[{n}]"] / 3, 2) for n in range(4)],
          "bf16 (two of three invocations)", [round(tmb[f"ttm_kernel[{n}]"] / 3, 2) for n in range(4)], flush=True)
    assert abs(bf[-1] - fits[-1]) <= 1e-5
    assert abs(bf[0] - fits[0]) <= 1e-2
