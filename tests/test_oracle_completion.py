"""Pins of the completion oracle: dense model values and central finite differences."""
import numpy as np
import pytest

import synth
from oracle import completion, ttm


def _small(seed=0, dims=(9, 8, 7), ranks=(3, 2, 4), n_obs=150):
    rng = np.random.default_rng(seed)
    idx = [rng.integers(0, L, n_obs).astype(np.int32) for L in dims]
    G = rng.standard_normal(ranks)
    F = [rng.standard_normal((L, K)) for L, K in zip(dims, ranks)]
    vals = rng.standard_normal(n_obs)
    return idx, G, F, vals


def test_model_values_match_dense_reconstruction():
    idx, G, F, _ = _small()
    R = G
    for n in range(3):
        R = ttm.ttm(R, F[n], n)
    np.testing.assert_allclose(completion.model_values(G, F, idx), R[tuple(idx)], rtol=1e-12, atol=1e-12)


def test_gradient_central_differences():
    idx, G, F, vals = _small(1)
    dG, dF = completion.gradient(G, F, idx, vals)
    h = 1e-6
    for c in np.ndindex(G.shape):
        Gp, Gm = G.copy(), G.copy()
        Gp[c] += h
        Gm[c] -= h
        fd = (completion.loss(Gp, F, idx, vals) - completion.loss(Gm, F, idx, vals)) / (2 * h)
        assert dG[c] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    rng = np.random.default_rng(2)
    for n in range(3):
        for _ in range(12):
            i, k = rng.integers(0, F[n].shape[0]), rng.integers(0, F[n].shape[1])
            Fp = [f.copy() for f in F]
            Fm = [f.copy() for f in F]
            Fp[n][i, k] += h
            Fm[n][i, k] -= h
            fd = (completion.loss(G, Fp, idx, vals) - completion.loss(G, Fm, idx, vals)) / (2 * h)
            assert dF[n][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_directional_derivative():
    idx, G, F, vals = _small(3)
    dG, dF = completion.gradient(G, F, idx, vals)
    rng = np.random.default_rng(4)
    for _ in range(4):
        DG = rng.standard_normal(G.shape)
        DF = [rng.standard_normal(f.shape) for f in F]
        h = 1e-6
        lp = completion.loss(G + h * DG, [f + h * d for f, d in zip(F, DF)], idx, vals)
        lm = completion.loss(G - h * DG, [f - h * d for f, d in zip(F, DF)], idx, vals)
        fd = (lp - lm) / (2 * h)
        an = np.sum(dG * DG) + sum(np.sum(a * b) for a, b in zip(dF, DF))
        assert an == pytest.approx(fd, rel=1e-6)


def test_completion_generator_is_seeded_and_noise_scaled():
    a = synth.make_completion((20, 15, 10), 4000, (3, 2, 2), noise=0.05, seed=7)
    b = synth.make_completion((20, 15, 10), 4000, (3, 2, 2), noise=0.05, seed=7)
    for x, y in zip(a["idx"], b["idx"]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a["noise"], b["noise"])
    assert abs(np.std(a["noise"]) - 0.05) < 0.005
    assert all(i.min() >= 0 and i.max() < L for i, L in zip(a["idx"], (20, 15, 10)))
