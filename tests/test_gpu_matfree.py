"""The matrix-free SVD step (block Krylov on Y itself, X -> Y^T (Y X), never
forming the Gram; Section 3 "SVD Component") against the FP64 oracle's HOOI,
and against the Gram route on the same tensor: wide Khat on four modes
(ranks 10, Khat = 1000) and ranks above 16 (K = 20, the 32-column block).
The matrix-free factors are held to Wedin's bound for a perturbation of Y of
its FP32 rounding (they never square Y), the Gram route's to its own."""
import numpy as np
import pytest

import synth
from oracle import coo, hooi, ttm
from tests.gpu_common import factor_tolerance, factor_tolerance_y, fit_noise

pytestmark = pytest.mark.gpu

CASES = {"4mode_k10": ((1500, 1000, 400, 60), 120_000, (0.9, 1.1, 1.3, 0.7), (10, 10, 10, 10), 2),
         "3mode_k20": ((1200, 900, 600), 150_000, (1.0, 1.1, 1.2), (20, 20, 20), 2),
         # Khat = 4096: W of the factor step no longer fits in LDS (tall-skinny product route)
         "4mode_k16": ((400, 300, 150, 60), 12_000, (0.9, 1.0, 1.1, 0.8), (16, 16, 16, 16), 1)}


def _run(tk, idx, vals, dims, ranks, F0, iters, method):
    ctx = tk.TuckerContext(0, eig_method=method)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals, np.float32), dims)
    ctx.set_ranks(ranks)
    for n, F in enumerate(F0):
        ctx.set_factor(n, np.ascontiguousarray(F))
    before = ctx.counters()
    fits = ctx.hooi_iterate(iters)
    after = ctx.counters()
    return ctx, fits, {k: after[k] - before[k] for k in after}


@pytest.mark.parametrize("name", list(CASES))
def test_matfree_hooi_matches_oracle_and_gram_route(tk, name):
    dims, nnz, zipf, ranks, iters = CASES[name]
    idx, vals = synth.make_tensor(dims, nnz, "zipf", zipf, "lognormal", seed=97)
    F0 = synth.orthonormal_init(9797, dims, ranks)
    ctx, fits, cnt = _run(tk, idx, vals, dims, ranks, F0, iters, "matfree")
    print(name, "matrix-free fits", fits, "counters", cnt, flush=True)
    assert cnt["eig_krylov_solves"] >= len(dims) * iters     # every mode took the Krylov route
    ctx_g, fits_g, _ = _run(tk, idx, vals, dims, ranks, F0, iters, "gram")
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    o = hooi.hooi(ic, vc, dims, F0, ranks, iters)
    print(name, "gram-route fits", fits_g, "oracle", o["fits"], flush=True)
    for a, b, g in zip(fits, o["fits"], fits_g):
        assert abs(a - b) <= max(1e-5, fit_noise(b))
        assert abs(a - g) <= max(1e-5, fit_noise(b))
    for n in range(len(dims)):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(ranks[n]), atol=1e-12)
        sv = np.linalg.svd(ttm.ttm_chain(ic, vc, o["factors"], n, dims), compute_uv=False)
        allowed = factor_tolerance_y(sv, ranks[n])
        allowed_g, _ = factor_tolerance(sv, ranks[n])
        d = hooi.projector_distance(F, o["factors"][n])
        dg = hooi.projector_distance(ctx_g.get_factor(n), o["factors"][n])
        print(f"  mode {n}: matrix-free vs oracle {d:.2e} (allowed {allowed:.2e}), Gram route vs oracle "
              f"{dg:.2e}", flush=True)
        assert d <= allowed
        assert dg <= allowed_g


def test_matfree_small_khat_takes_gram_route(tk):
    # Khat = 100 < 192: the option falls back to the Gram route (dense solver)
    dims, ranks = (300, 200, 100), (10, 10, 10)
    idx, vals = synth.make_tensor(dims, 20_000, "zipf", (1.1, 1.1, 1.1), "lognormal", seed=98)
    F0 = synth.orthonormal_init(9898, dims, ranks)
    _, fits, cnt = _run(tk, idx, vals, dims, ranks, F0, 1, "matfree")
    assert cnt["eig_krylov_solves"] == 0
    _, fits_g, _ = _run(tk, idx, vals, dims, ranks, F0, 1, "gram")
    assert fits == fits_g
