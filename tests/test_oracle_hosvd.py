"""Pins of the HOSVD initialisation oracle (Section 1 "HOOI Procedure",
Section 2.2): the dense definition against an eigendecomposition of the
unfolding's Gram and a rank-one tensor; the sketched range finder against the
dense definition where it must be exact (multilinear rank at most K, and
identity sketches for any tensor)."""
import numpy as np

from oracle import hooi, hosvd


def _sin(U, V):
    """||(I - U U^T) V||_F for orthonormal U, V: the sines of the principal
    angles, computed without the cancellation of the projector difference."""
    return float(np.linalg.norm(V - U @ (U.T @ V)))


def _as_coo(T):
    grids = np.meshgrid(*[np.arange(L) for L in T.shape], indexing="ij")
    return [g.ravel().astype(np.int32) for g in grids], T.ravel()


def _low_rank(dims, r, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(r)
    A = [rng.standard_normal((L, k)) for L, k in zip(dims, r)]
    return np.einsum("abc,ia,jb,kc->ijk", G, *A)


def test_dense_hosvd_matches_gram_eigenvectors():
    rng = np.random.default_rng(1)
    T = rng.standard_normal((7, 6, 5)) + 3.0 * _low_rank((7, 6, 5), (1, 1, 1), 2)
    F = hosvd.hosvd_dense(T, (2, 3, 2))
    for n, K in enumerate((2, 3, 2)):
        Tn = np.moveaxis(T, n, 0).reshape(T.shape[n], -1)
        w, V = np.linalg.eigh(Tn @ Tn.T)
        assert _sin(F[n], V[:, ::-1][:, :K]) < 1e-12


def test_dense_hosvd_of_rank_one_tensor():
    a, b, c = np.array([1.0, 2.0, 2.0]), np.array([0.0, 3.0, 4.0, 0.0]), np.array([1.0, -1.0])
    T = np.einsum("i,j,k->ijk", a, b, c)
    F = hosvd.hosvd_dense(T, (1, 1, 1))
    for f, v in zip(F, (a, b, c)):
        np.testing.assert_allclose(np.abs(f[:, 0]), np.abs(v) / np.linalg.norm(v), atol=1e-14)


def test_sketched_is_exact_for_low_multilinear_rank():
    dims, r = (9, 8, 7), (2, 3, 2)
    T = _low_rank(dims, r, 3)
    idx, vals = _as_coo(T)
    rng = np.random.default_rng(4)
    sk = [rng.standard_normal((L, k)) for L, k in zip(dims, r)]
    F, s = hosvd.hosvd_sketched(idx, vals, dims, sk, r)
    Fd = hosvd.hosvd_dense(T, r)
    for n in range(3):
        assert _sin(F[n], Fd[n]) < 1e-12
        np.testing.assert_allclose(F[n].T @ F[n], np.eye(r[n]), atol=1e-12)


def test_sketched_with_identity_sketches_is_the_hosvd_of_any_tensor():
    rng = np.random.default_rng(5)
    dims, K = (6, 5, 4), (2, 2, 3)
    T = rng.standard_normal(dims)
    idx, vals = _as_coo(T)
    F, _ = hosvd.hosvd_sketched(idx, vals, dims, [np.eye(L) for L in dims], K)
    Fd = hosvd.hosvd_dense(T, K)
    for n in range(3):
        assert _sin(F[n], Fd[n]) < 1e-12


def test_sketch_narrower_than_the_rank_misses_the_range():
    # a one-column sketch of a mode of rank 3 cannot see its whole range:
    # the check above is sharp enough to notice
    dims, r = (9, 8, 7), (3, 3, 3)
    T = _low_rank(dims, r, 6)
    idx, vals = _as_coo(T)
    rng = np.random.default_rng(7)
    sk = [rng.standard_normal((L, 1)) for L in dims]
    F, _ = hosvd.hosvd_sketched(idx, vals, dims, sk, (1, 1, 1))
    Fd = hosvd.hosvd_dense(T, (1, 1, 1))
    assert max(_sin(F[n], Fd[n]) for n in range(3)) > 1e-3
