"""HOSVD initialisation (tk_init_hosvd) against the oracle: the factors are
the leading left singular vectors of T_(n) times the Kronecker product of
caller-drawn Gaussian sketches (Section 1 "HOOI Procedure", Section 2.2).
Exact for a tensor of low multilinear rank (the truncated HOSVD from the dense
unfoldings); on sparse Zipf tensors the GPU factors match the FP64 oracle's
to 1e-5 where the spectrum separates the leading subspace (a sin-theta bound
otherwise), and the fit of the initial decomposition to the FP32 noise."""
import numpy as np
import pytest

import synth
from oracle import coo, hooi, hosvd, ttm
from tests.gpu_common import factor_tolerance, fit_noise, zipf_tensor

pytestmark = pytest.mark.gpu


def _sketches(dims, ranks, seed):
    return synth.gaussian_factors(seed, dims, ranks)


def _ctx(tk, idx, vals, dims, ranks):
    ctx = tk.TuckerContext(0)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals, np.float32), dims)
    ctx.set_ranks(ranks)
    return ctx


def test_hosvd_exact_for_low_multilinear_rank(tk):
    dims, r = (40, 30, 20), (3, 3, 3)
    rng = np.random.default_rng(12)
    G = rng.standard_normal(r)
    A = [rng.standard_normal((L, k)) for L, k in zip(dims, r)]
    T = np.einsum("abc,ia,jb,kc->ijk", G, *A).astype(np.float32)
    grids = np.meshgrid(*[np.arange(L) for L in dims], indexing="ij")
    idx = [g.ravel().astype(np.int32) for g in grids]
    ctx = _ctx(tk, idx, T.ravel(), dims, r)
    fit = ctx.init_hosvd(_sketches(dims, r, 81))
    Fd = hosvd.hosvd_dense(T.astype(np.float64), r)
    for n in range(3):
        Fg = ctx.get_factor(n)
        np.testing.assert_allclose(Fg.T @ Fg, np.eye(r[n]), atol=1e-12)
        d = float(np.linalg.norm(Fd[n] - Fg @ (Fg.T @ Fd[n])))
        print(f"mode {n}: sin distance from the dense HOSVD {d:.2e}", flush=True)
        assert d <= 1e-5
    # the decomposition is exact up to FP32 rounding: ||T||^2 - ||G||^2 ~ u ||T||^2
    assert fit >= 1.0 - 2e-3


@pytest.mark.parametrize("name", ["c1", "zipf"])
def test_hosvd_matches_oracle(tk, name):
    if name == "c1":
        w = synth.make_workload("c1")
        idx, vals, dims, ranks = w["idx"], w["vals"], w["dims"], w["ranks"]
    else:
        dims, ranks = (2000, 1000, 400), (10, 10, 10)
        idx, vals = zipf_tensor(dims, 100_000, s=1.1, seed=83)
    sk = _sketches(dims, ranks, 84)
    ctx = _ctx(tk, idx, vals, dims, ranks)
    fit = ctx.init_hosvd(sk)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    Fo, _ = hosvd.hosvd_sketched(ic, vc, dims, sk, ranks)
    for n in range(len(dims)):
        Fg = ctx.get_factor(n)
        np.testing.assert_allclose(Fg.T @ Fg, np.eye(ranks[n]), atol=1e-12)
        sv = np.linalg.svd(ttm.ttm_chain(ic, vc, sk, n, dims), compute_uv=False)
        allowed, cond = factor_tolerance(sv, ranks[n])
        d = hooi.projector_distance(Fg, Fo[n])
        print(f"{name} mode {n}: projector distance {d:.2e} (allowed {allowed:.2e})", flush=True)
        assert d <= allowed
    v = np.asarray(vc, np.float64)
    G = hooi.core(ic, vc, Fo)
    fit_o = hooi.fit_from_norms(float(v @ v), float(np.sum(G * G)))
    print(f"{name}: fit after the HOSVD {fit:.8f}, oracle {fit_o:.8f}", flush=True)
    assert abs(fit - fit_o) <= fit_noise(fit_o)
    # HOOI continues from it (Gauss-Seidel: non-decreasing within noise)
    fits = ctx.hooi_iterate(2)
    assert fits[0] >= fit - fit_noise(fit)
    assert fits[1] >= fits[0] - fit_noise(fits[0])


def test_hosvd_requires_ranks_and_shapes(tk):
    idx, vals = zipf_tensor((50, 40, 30), 2000, s=1.1, seed=85)
    ctx = tk.TuckerContext(0)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], vals, (50, 40, 30))
    with pytest.raises(tk.TuckerError, match="STATE"):
        ctx._check(ctx._L.tk_init_hosvd(ctx._h, None, 0, None))
    ctx.set_ranks((3, 3, 3))
    with pytest.raises(tk.TuckerError, match="INVALID_ARG"):
        ctx._check(ctx._L.tk_init_hosvd(ctx._h, None, 0, None))
    with pytest.raises(ValueError):
        ctx.init_hosvd([np.zeros((50, 3)), np.zeros((40, 3))])
