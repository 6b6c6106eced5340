"""Pins of the HOOI oracle (Section 2.2): LAPACK SVD, orthonormality, exact
reconstruction at full rank, the core identities and a non-decreasing fit."""
import numpy as np
import pytest

import synth
from oracle import coo, hooi, ttm


def test_svd_step_matches_lapack_svd():
    rng = np.random.default_rng(0)
    for rows, cols, K in [(50, 12, 4), (8, 20, 3), (30, 30, 30)]:
        Z = rng.standard_normal((rows, cols)) @ np.diag(np.linspace(3, 0.1, cols))
        U, s, nv = hooi.leading_left_singular_vectors(Z, K)
        U2, s2, _ = np.linalg.svd(Z, full_matrices=False)
        k = min(K, nv)
        np.testing.assert_allclose(s[:k], s2[:k], rtol=1e-12)
        assert hooi.projector_distance(U[:, :k], U2[:, :k]) < 1e-10
        np.testing.assert_allclose(U.T @ U, np.eye(K), atol=1e-12)


def test_svd_step_completes_rank_deficient():
    Z = np.zeros((6, 4))
    Z[1, 0] = 2.0
    Z[3, 2] = 1.0
    U, s, nv = hooi.leading_left_singular_vectors(Z, 4)
    assert nv == 2
    np.testing.assert_allclose(U.T @ U, np.eye(4), atol=1e-14)
    assert abs(abs(U[1, 0]) - 1) < 1e-14 and abs(abs(U[3, 1]) - 1) < 1e-14


def _dense_filled(dims, seed):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(L) for L in dims], indexing="ij")
    idx = [g.ravel() for g in grids]
    vals = rng.standard_normal(len(idx[0])).astype(np.float32)
    return coo.coalesce(idx, vals)


def test_full_rank_reconstruction_is_exact():
    dims = (4, 3, 5)
    idx, vals, nsq = _dense_filled(dims, 1)
    F0 = synth.orthonormal_init(7, dims, dims)
    out = hooi.hooi(idx, vals, dims, F0, dims, iters=1)
    G = out["core"]
    assert out["fits"][-1] == pytest.approx(1.0, abs=1e-7)
    assert np.sum(G * G) == pytest.approx(nsq, rel=1e-12)
    R = G
    for n in range(3):
        R = ttm.ttm(R, out["factors"][n], n)
    np.testing.assert_allclose(R, ttm.dense(idx, vals, dims), atol=1e-12)


def test_core_definition_matches_dense_ttms_and_last_mode_identity():
    rng = np.random.default_rng(2)
    dims, ranks = (7, 6, 5), (3, 2, 4)
    idx, vals, _ = coo.coalesce([rng.integers(0, L, 80) for L in dims], rng.standard_normal(80))
    F0 = synth.orthonormal_init(3, dims, ranks)
    out = hooi.hooi(idx, vals, dims, F0, ranks, iters=2, record=True)
    F = out["factors"]
    T = ttm.dense(idx, vals, dims)
    G = T
    for n in range(3):
        G = ttm.ttm(G, F[n].T, n)
    np.testing.assert_allclose(out["core"], G, atol=1e-12)
    # Gauss-Seidel: G_(N) = F_N^T Z_(N), where Z_(N) came from the latest factors
    n_last, Z_last, F_last = out["history"][-1]
    assert n_last == 2
    np.testing.assert_allclose(ttm.unfold(out["core"], 2), F_last.T @ Z_last, atol=1e-12)
    # ||G||^2 = sum of the K_N largest squared singular values of Z_(N)
    s = np.linalg.svd(Z_last, compute_uv=False)
    assert np.sum(out["core"] ** 2) == pytest.approx(np.sum(s[:ranks[2]] ** 2), rel=1e-12)
    # fit formula equals the dense residual
    Rec = out["core"]
    for n in range(3):
        Rec = ttm.ttm(Rec, F[n], n)
    fit_dense = 1 - np.linalg.norm(T - Rec) / np.linalg.norm(T)
    assert out["fits"][-1] == pytest.approx(fit_dense, abs=1e-10)


def test_factors_orthonormal_and_fit_non_decreasing_c1():
    w = synth.make_workload("c1")
    idx, vals, nsq = coo.coalesce(w["idx"], w["vals"])
    out = hooi.hooi(idx, vals, w["dims"], w["F0"], w["ranks"], iters=3)
    for F in out["factors"]:
        np.testing.assert_allclose(F.T @ F, np.eye(F.shape[1]), atol=1e-12)
    fits = out["fits"]
    for a, b in zip(fits, fits[1:]):
        assert b >= a - 1e-12 * max(1.0, abs(a))
    assert 0.0 < fits[-1] < 1.0


def test_jacobi_sweep_uses_input_factors():
    rng = np.random.default_rng(9)
    dims, ranks = (8, 7, 6), (2, 3, 2)
    idx, vals, _ = coo.coalesce([rng.integers(0, L, 100) for L in dims], rng.standard_normal(100))
    F0 = synth.orthonormal_init(1, dims, ranks)
    out = hooi.hooi(idx, vals, dims, F0, ranks, iters=1, sweep="jacobi")
    Z1 = ttm.ttm_chain(idx, vals, F0, 1, dims)      # mode 2 with the *input* factors
    U, _, _ = hooi.leading_left_singular_vectors(Z1, ranks[1])
    assert hooi.projector_distance(out["factors"][1], U) < 1e-12


def test_projector_distance_is_rotation_free():
    rng = np.random.default_rng(4)
    U, _ = np.linalg.qr(rng.standard_normal((20, 4)))
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    assert hooi.projector_distance(U @ Q, U) < 1e-14
    V, _ = np.linalg.qr(rng.standard_normal((20, 4)))
    assert hooi.projector_distance(V, U) > 0.1
