"""The C ABI's failure contract, checkpoint/resume, and two paths that only
run under particular inputs (the rerun of modes after a rank-deficient mode,
the dense fallback of the block-Krylov eigensolve), through the C ABI.

Failures are forced from the host: a memory limit below the plan, completion
switched off for a rank-deficient penultimate matrix, ranks outside what the
build handles, calls out of order.  No kernel is made to fail."""
import numpy as np
import pytest

import synth
from oracle import coo, hooi
from tests.gpu_common import factor_tolerance, rel_fro, zipf_tensor

pytestmark = pytest.mark.gpu


def _ctx(tk, idx, vals, dims, ranks=None, **opt):
    ctx = tk.TuckerContext(0, **opt)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals, np.float32), dims)
    if ranks is not None:
        ctx.set_ranks(ranks)
    return ctx


def test_mem_limit_gives_oom_before_allocating(tk):
    idx, vals = zipf_tensor((3000, 2000, 500), 100_000, s=1.1, seed=81)
    dims = (3000, 2000, 500)
    ctx = _ctx(tk, idx, vals, dims)
    ctx.set_options(mem_limit_bytes=1 << 20)          # 1 MiB: the plan needs far more
    with pytest.raises(tk.TuckerError, match="OOM"):
        ctx.set_ranks((10, 10, 10))
    with pytest.raises(tk.TuckerError, match="STATE"):
        ctx.hooi_iterate(1)                            # no plan was kept
    ctx.set_options(mem_limit_bytes=0)
    ctx.set_ranks((10, 10, 10))                        # and the context is still usable
    assert len(ctx.hooi_iterate(1)) == 1
    # a load whose device copies exceed the limit fails the same way
    small = tk.TuckerContext(0, mem_limit_bytes=4096)
    with pytest.raises(tk.TuckerError, match="OOM"):
        small.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals), dims)


def _rank_deficient_tensor():
    # mode-0 unfolding of rank 1 over 8 nonempty slices (K_0 = 3); modes 1 and
    # 2 have empty slices (indices 6-8 and 5-6 never occur).  Small integers, so
    # every product is exact in FP32 and the unfolding is exactly rank 1.
    rng = np.random.default_rng(5)
    a = rng.integers(1, 9, 8).astype(np.float64)
    B = rng.integers(-4, 5, (6, 5)).astype(np.float64)
    B[B == 0] = 1.0
    i0, i1, i2 = np.meshgrid(np.arange(8), np.arange(6), np.arange(5), indexing="ij")
    idx = [i0.ravel().astype(np.int32), i1.ravel().astype(np.int32), i2.ravel().astype(np.int32)]
    vals = (a[i0] * B[i1, i2]).ravel().astype(np.float32)
    return idx, vals, (10, 9, 7), (3, 2, 2)


def test_rank_deficient_numeric_error_when_completion_off(tk):
    idx, vals, dims, ranks = _rank_deficient_tensor()
    ctx = _ctx(tk, idx, vals, dims, ranks, complete_rank_deficient=0)
    F0 = synth.orthonormal_init(11, dims, ranks)
    for n in range(3):
        ctx.set_factor(n, F0[n])
    with pytest.raises(tk.TuckerError, match="NUMERIC"):
        ctx.hooi_iterate(1)


def test_rank_deficient_mode_reruns_clear_empty_slice_rows(tk):
    """Mode 0 fails inside a Gauss-Seidel invocation; modes 1 and 2 run again
    after its completion.  Their factors must be zero on the rows of empty
    slices (the input factors are not), orthonormal, and equal to the
    oracle's subspaces."""
    idx, vals, dims, ranks = _rank_deficient_tensor()
    ctx = _ctx(tk, idx, vals, dims, ranks)
    F0 = synth.orthonormal_init(11, dims, ranks)
    for n in range(3):
        ctx.set_factor(n, F0[n])
    fits = ctx.hooi_iterate(2)
    o = hooi.hooi(idx, vals.astype(np.float64), dims, F0, ranks, 2)
    for n in range(3):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(ranks[n]), atol=1e-12)
    assert np.all(ctx.get_factor(1)[6:] == 0.0) and np.all(ctx.get_factor(2)[5:] == 0.0)
    assert hooi.projector_distance(ctx.get_factor(0)[:, :1], o["factors"][0][:, :1]) <= 1e-5
    for n in (1, 2):
        assert hooi.projector_distance(ctx.get_factor(n), o["factors"][n]) <= 1e-5, n
    np.testing.assert_allclose(fits, o["fits"], atol=1e-6)


def test_unsupported_and_invalid_arguments(tk):
    idx, vals = zipf_tensor((300, 200, 100), 5_000, s=1.1, seed=82)
    dims = (300, 200, 100)
    ctx = _ctx(tk, idx, vals, dims)
    with pytest.raises(tk.TuckerError, match="UNSUPPORTED"):
        ctx.set_ranks((65, 10, 10))                    # ranks above 64
    with pytest.raises(tk.TuckerError, match="INVALID_ARG"):
        ctx.set_ranks((10, 10, 101))                   # K_n > L_n
    with pytest.raises(tk.TuckerError, match="INVALID_ARG"):
        ctx.load_coo([i for i in idx] * 3, vals, dims * 3)   # N = 9
    with pytest.raises(tk.TuckerError, match="STATE"):
        ctx.ttm_chain(0)                               # no ranks set


def test_checkpoint_resume_bit_identical(tk):
    """The HOOI state is the decomposition: k invocations, the factors saved
    and loaded into a fresh context over the same tensor, then I - k more,
    equal I invocations in one context bit for bit."""
    w = synth.make_workload("c2", scale=0.002)
    dims, ranks = w["dims"], w["ranks"]
    a = _ctx(tk, w["idx"], w["vals"], dims, ranks)
    for n, F in enumerate(w["F0"]):
        a.set_factor(n, np.ascontiguousarray(F))
    straight = a.hooi_iterate(4)
    b = _ctx(tk, w["idx"], w["vals"], dims, ranks)
    for n, F in enumerate(w["F0"]):
        b.set_factor(n, np.ascontiguousarray(F))
    first = b.hooi_iterate(2)
    saved = [b.get_factor(n) for n in range(3)]
    del b
    c = _ctx(tk, w["idx"], w["vals"], dims, ranks)
    for n in range(3):
        c.set_factor(n, saved[n])
    rest = c.hooi_iterate(2)
    assert first + rest == straight
    for n in range(3):
        np.testing.assert_array_equal(c.get_factor(n), a.get_factor(n))
    ca, fa = a.core()
    cc, fc = c.core()
    np.testing.assert_array_equal(ca, cc)
    assert fa == fc


def test_krylov_dense_fallback_matches_oracle(tk):
    """Khat = 216 takes the block-Krylov eigensolve.  With eig_tol far below
    any reachable error estimate every solve falls back to the dense solver;
    the result still matches the oracle, and the counters show the
    fallbacks.  With the default tolerance no solve falls back here."""
    dims, ranks = (300, 200, 120, 60), (6, 6, 6, 6)
    idx, vals = synth.make_tensor(dims, 40_000, "zipf", (0.9, 1.1, 1.3, 0.7), "lognormal", seed=41)
    F0 = synth.orthonormal_init(41 + 7690, dims, ranks)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    o = hooi.hooi(ic, vc, dims, F0, ranks, 2)
    for tol, expect_fallback in ((1e-30, True), (0.0, False)):
        ctx = _ctx(tk, idx, vals, dims, ranks, eig_tol=tol)
        for n, F in enumerate(F0):
            ctx.set_factor(n, np.ascontiguousarray(F))
        fits = ctx.hooi_iterate(2)
        cnt = ctx.counters()
        print("eig_tol", tol, "fits", fits, "oracle", o["fits"], cnt, flush=True)
        assert cnt["eig_krylov_solves"] == 8
        if expect_fallback:
            assert cnt["eig_dense_fallbacks"] == 8
        else:
            assert cnt["eig_dense_fallbacks"] == 0
        for a, b in zip(fits, o["fits"]):
            assert abs(a - b) <= 1e-5
        from oracle import ttm
        for n in range(4):
            sv = np.linalg.svd(ttm.ttm_chain(ic, vc, o["factors"], n, dims), compute_uv=False)
            allowed, _ = factor_tolerance(sv, ranks[n])
            assert hooi.projector_distance(ctx.get_factor(n), o["factors"][n]) <= allowed


def test_torch_allocator_hook(tk):
    """With torch's caching allocator behind the context's device memory the
    results are the same bit for bit, and the memory shows up in torch's
    accounting while the context lives."""
    import torch
    w = synth.make_workload("c2", scale=0.001)
    dims, ranks = w["dims"], w["ranks"]
    base = torch.cuda.memory_allocated()
    a = tk.TuckerContext(0, allocator="torch")
    a.load_coo([np.ascontiguousarray(i, np.int32) for i in w["idx"]], np.ascontiguousarray(w["vals"]), dims)
    a.set_ranks(ranks)
    for n, F in enumerate(w["F0"]):
        a.set_factor(n, np.ascontiguousarray(F))
    fa = a.hooi_iterate(2)
    assert torch.cuda.memory_allocated() > base
    b = _ctx(tk, w["idx"], w["vals"], dims, ranks)
    for n, F in enumerate(w["F0"]):
        b.set_factor(n, np.ascontiguousarray(F))
    assert b.hooi_iterate(2) == fa
    a.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
