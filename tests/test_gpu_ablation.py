"""The partition ablations against the oracle: CoarseG bins (Section 5, whole
slices in a random order, contiguous blocks) must match the oracle's
assignment bit for bit; the TTM-chain on CoarseG bins, with the vector-ALU
kernel forced on Lite bins, with the fiber-factored kernel, and without a
partition (atomics) must match the FP64 oracle's Y to 1e-5."""
import numpy as np
import pytest

import synth
from oracle import coo, lite
from tests.gpu_common import oracle_Y, rel_fro, zipf_tensor

pytestmark = pytest.mark.gpu


def _ctx(tk, idx, vals, dims, **opt):
    ctx = tk.TuckerContext(0, **opt)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals, np.float32), dims)
    return ctx


CASES = {"zipf11": (lambda: zipf_tensor((5000, 3000, 800), 200_000, s=1.1, seed=51), (10, 10, 10), 448),
         "zipf15": (lambda: zipf_tensor((5000, 3000, 800), 200_000, s=1.5, seed=52), (10, 10, 10), 448),
         "4mode": (lambda: zipf_tensor((600, 500, 200, 40), 40_000, s=(0.9, 1.1, 1.3, 0.7), seed=53),
                   (10, 10, 10, 10), 1024)}


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_partition_and_ttm(tk, name):
    make, ranks, wg = CASES[name]
    idx, vals = make()
    dims = tuple(int(i.max()) + 1 for i in idx)
    print("case", name, dims, len(vals), flush=True)
    ctx = _ctx(tk, idx, vals, dims, partition="coarse", wg_nnz_target=wg)
    orders = [synth.permutation(61, 700 + n, L) for n, L in enumerate(dims)]
    for n in range(len(dims)):
        ctx.set_slice_order(n, orders[n])
    ctx.set_ranks(ranks)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    F = [synth.normal(77, 200 + n, d * k).reshape(d, k) for n, (d, k) in enumerate(zip(dims, ranks))]
    F32 = [f.astype(np.float32).astype(np.float64) for f in F]
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    for n in range(len(dims)):
        g = ctx.partition(n)
        st = g["stats"]
        o = lite.partition_mode(ic[n], dims[n], st["P"], coarse_order=orders[n])
        np.testing.assert_array_equal(g["bin_ptr"], o.bin_ptr)
        np.testing.assert_array_equal(g["elem_order"], o.elem_order)
        np.testing.assert_array_equal(g["seg_bin"], o.seg_bin)
        np.testing.assert_array_equal(g["seg_slice"], o.seg_slice)
        np.testing.assert_array_equal(g["seg_begin"][:-1], o.seg_begin)
        np.testing.assert_array_equal(g["seg_bad"], o.seg_bad)
        for k in ("P", "m", "L_nonempty", "E_max", "R_sum", "R_max", "n_bad"):
            assert st[k] == o.stats[k], k
        assert st["n_bad"] == 0 and st["R_sum"] == st["L_nonempty"]
        Y, rows = ctx.ttm_chain(n)
        Yo, rows_o = oracle_Y(ic, vc, F32, n, dims)
        np.testing.assert_array_equal(rows, rows_o)
        err = rel_fro(Y, Yo)
        print(f"  mode {n}: CoarseG E_max={st['E_max']} R_max={st['R_max']} rel err {err:.2e}", flush=True)
        assert err <= 1e-5
        Y2, _ = ctx.ttm_chain(n)
        np.testing.assert_array_equal(Y, Y2)


@pytest.mark.parametrize("kernel", ["vector", "atomic", "fiber"])
@pytest.mark.parametrize("name", ["zipf15", "4mode"])
def test_ttm_kernel_choices(tk, kernel, name):
    make, ranks, wg = CASES[name]
    idx, vals = make()
    dims = tuple(int(i.max()) + 1 for i in idx)
    ctx = _ctx(tk, idx, vals, dims, ttm_kernel=kernel, wg_nnz_target=wg)
    ctx.set_ranks(ranks)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    F = [synth.normal(78, 200 + n, d * k).reshape(d, k) for n, (d, k) in enumerate(zip(dims, ranks))]
    F32 = [f.astype(np.float32).astype(np.float64) for f in F]
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    for n in range(len(dims)):
        Y, rows = ctx.ttm_chain(n)
        Yo, rows_o = oracle_Y(ic, vc, F32, n, dims)
        np.testing.assert_array_equal(rows, rows_o)
        err = rel_fro(Y, Yo)
        print(f"{kernel} mode {n}: rel err {err:.2e}", flush=True)
        assert err <= 1e-5


FIBER_CASES = {
    # long fibers: the last remaining mode has few ids, odd ranks
    "4mode_long": (lambda: zipf_tensor((200, 100, 50, 8), 60_000, s=(1.0, 0.9, 0.8, 0.5), seed=54), (3, 5, 7, 6)),
    "3mode_long": (lambda: zipf_tensor((3000, 400, 6), 80_000, s=(1.2, 1.0, 0.5), seed=55), (16, 9, 5)),
    "4mode_k16": (lambda: zipf_tensor((300, 200, 60, 30), 30_000, s=(0.9, 1.1, 1.3, 0.7), seed=56), (16, 16, 16, 16)),
}


@pytest.mark.parametrize("name", list(FIBER_CASES))
def test_fiber_kernel_matches_oracle_and_reruns_bit_identical(tk, name):
    make, ranks = FIBER_CASES[name]
    idx, vals = make()
    dims = tuple(int(i.max()) + 1 for i in idx)
    ctx = _ctx(tk, idx, vals, dims, ttm_kernel="fiber")
    ctx.set_ranks(ranks)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    F = [synth.normal(79, 200 + n, d * k).reshape(d, k) for n, (d, k) in enumerate(zip(dims, ranks))]
    F32 = [f.astype(np.float32).astype(np.float64) for f in F]
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    for n in range(len(dims)):
        Y, rows = ctx.ttm_chain(n)
        Yo, rows_o = oracle_Y(ic, vc, F32, n, dims)
        np.testing.assert_array_equal(rows, rows_o)
        err = rel_fro(Y, Yo)
        st = ctx.partition_stats(n)
        print(f"{name} fiber mode {n}: rel err {err:.2e}, split slices {st['n_bad']}", flush=True)
        assert err <= 1e-5
        Y2, _ = ctx.ttm_chain(n)
        np.testing.assert_array_equal(Y, Y2)
