"""Parity at the largest one-GPU workload, in the configuration the benchmark
times: 4,000,000 x 4,000,000 x 2,000,000, 4.0e9 draws (Zipf 0.8 / 1.2 / 1.5),
lognormal values, ranks 10, streamed into the library in chunks.

The oracle cannot hold or run the whole workload, so in the same pass over the
drawn chunks that feeds the GPU it computes, from the draws (never from the
library's outputs), with its C++/OpenMP FP64 code:
  * the merged cardinality of every slice of every mode (distinct
    coordinates), hence m' and Lite's statistics and segments (bit-exact);
  * the merged values of 3,000 sampled coordinates (bit-exact);
  * rows of Y_(n) for about 1,000 seeded slices per mode: the 500 heaviest
    Zipf ranks (the ten heaviest among them, and the slices Lite splits
    across bins) and 500 random ids.
HOOI at this size is checked by properties (orthonormal factors, fit within
rounding noise of non-decreasing, bit-identical rerun)."""
import numpy as np
import pytest

import synth
from oracle import cpp
from tests.gpu_common import fit_noise, rel_fro

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

CHUNK = 1 << 27


@pytest.fixture(scope="module")
def c5(tk):
    import time
    import torch
    stream = synth.WorkloadStream("c5")
    dims, nnz = stream.dims, stream.nnz
    N = len(dims)
    F0 = stream.initial_factors()
    rng = np.random.default_rng(55)
    picks = []
    for n in range(N):
        heavy = stream.samplers[n].perm[:500]                 # Zipf ranks 1 .. 500
        picks.append(np.unique(np.concatenate([heavy, rng.choice(dims[n], 500, replace=False)])))
    accs = [cpp.RowAccumulator(F0, n, dims[n], picks[n]) for n in range(N)]
    dc = cpp.DistinctCounter(dims)
    pos = np.sort(rng.choice(nnz, 3000, replace=False))
    samp = np.stack([np.concatenate(stream.chunk(int(p), 1)[0]) for p in pos])     # (3000, N)
    samp = np.unique(samp, axis=0)
    ks = cpp.KeySums([samp[:, j] for j in range(N)], dims[0])
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
        dc.add(idx)
        ks.add(idx, vals)
        if (a // CHUNK) % 5 == 0:
            print(f"c5 chunk at {a}: {time.time() - t0:.0f}s", flush=True)
    ctx.load_end()
    print(f"c5 loaded on the GPU, {time.time() - t0:.0f}s", flush=True)
    m_o, sizes = dc.finish()
    merged_vals, merged_cnt = ks.finish()
    print(f"oracle: {m_o} distinct coordinates, {time.time() - t0:.0f}s", flush=True)
    ctx.set_ranks(stream.ranks)
    print(f"partition and layout built, {time.time() - t0:.0f}s", flush=True)
    return dict(stream=stream, ctx=ctx, F0=F0, picks=picks, accs=accs, m_o=m_o, sizes=sizes, samp=samp,
                merged_vals=merged_vals, merged_cnt=merged_cnt)


def test_c5_coalesce(c5):
    ctx = c5["ctx"]
    m, norm_sq = ctx.tensor_info()
    assert m == c5["m_o"]
    assert c5["stream"].nnz >= (1 << 31)   # draws beyond 32-bit signed element counts
    ic, vc = ctx.get_coo()
    # merged values of the sampled coordinates: canonical order is lexicographic,
    # so locate each one by nested binary searches
    samp = c5["samp"]
    got = np.empty(len(samp), np.float32)
    for k, c in enumerate(samp):
        a, b = np.searchsorted(ic[0], c[0], "left"), np.searchsorted(ic[0], c[0], "right")
        a, b = a + np.searchsorted(ic[1][a:b], c[1], "left"), a + np.searchsorted(ic[1][a:b], c[1], "right")
        i = a + np.searchsorted(ic[2][a:b], c[2], "left")
        assert i < b and ic[2][i] == c[2]
        got[k] = vc[i]
    assert np.all(c5["merged_cnt"] >= 1)
    np.testing.assert_array_equal(got, c5["merged_vals"])
    assert abs(norm_sq - float(np.dot(vc.astype(np.float64), vc.astype(np.float64)))) <= 1e-9 * norm_sq


def test_c5_partition(c5):
    ctx = c5["ctx"]
    for n in range(3):
        g = ctx.partition(n, elem_order=False)
        st = g["stats"]
        ost, sb, ss, sc, bad = cpp.lite(c5["sizes"][n], st["P"])
        np.testing.assert_array_equal(g["seg_bin"], sb)
        np.testing.assert_array_equal(g["seg_slice"], ss)
        np.testing.assert_array_equal(np.diff(g["seg_begin"]), sc)
        np.testing.assert_array_equal(g["seg_bad"], bad)
        for k in ("limit", "m", "L_nonempty", "n_stage1", "E_max", "R_sum", "R_max", "n_bad"):
            assert st[k] == ost[k], (n, k)
        assert st["E_max"] <= st["limit"]
        assert st["R_max"] <= -(-st["L_nonempty"] // st["P"]) + 2
        # the sampled slices include split ones
        split = set(np.asarray(g["seg_slice"])[np.asarray(g["seg_bad"]) == 1].tolist())
        assert len(split & set(c5["picks"][n].tolist())) >= 20
        print(f"mode {n}: P={st['P']} E_max={st['E_max']} R_max={st['R_max']} bad={st['n_bad']}", flush=True)


def test_c5_ttm_sampled_rows(c5):
    import torch
    ctx = c5["ctx"]
    for n, F in enumerate(c5["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    for n in range(3):
        Y, rows = ctx.ttm_chain(n, device=True)
        rows_h = rows.cpu().numpy()
        pick = c5["picks"][n]
        Yo = c5["accs"][n].rows
        present = np.isin(pick, rows_h)
        assert np.all(np.linalg.norm(Yo[~present], axis=1) == 0.0)   # empty slices: no row, zero in the oracle
        at = torch.from_numpy(np.searchsorted(rows_h, pick[present])).cuda()
        Yg = Y.index_select(0, at).double().cpu().numpy()
        Yo = Yo[present]
        err = rel_fro(Yg, Yo)
        row_err = np.linalg.norm(Yg - Yo, axis=1) / np.maximum(np.linalg.norm(Yo, axis=1), 1e-300)
        print(f"mode {n}: {present.sum()} sampled rows, rel err {err:.2e}, worst row {row_err.max():.2e}", flush=True)
        assert err <= 1e-5
        assert row_err.max() <= 1e-4
        del Y, rows


def test_c5_hooi_properties(c5):
    ctx = c5["ctx"]
    F0 = c5["F0"]

    def run(prec, iters):
        ctx.set_options(prec=prec, refine=1)
        for n, F in enumerate(F0):
            ctx.set_factor(n, np.ascontiguousarray(F))
        return ctx.hooi_iterate(iters)

    fits = run("fp32", 4)
    print("c5 fits fp32", fits, flush=True)
    for a, b in zip(fits, fits[1:]):
        assert b >= a - fit_noise(a)
    for n in range(3):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(10), atol=1e-12)
    assert run("fp32", 4) == fits
    bf = run("bf16", 4)
    print("c5 fits bf16-gram then refined", bf, flush=True)
    assert abs(bf[-1] - fits[-1]) <= 1e-5
