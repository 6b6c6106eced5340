"""Pins of the TTM-chain oracle (eq. 1, Appendix A) against dense definitions."""
import numpy as np
import pytest

from oracle import coo, ttm


def _random_sparse(rng, dims, m):
    idx = [rng.integers(0, L, m) for L in dims]
    vals = rng.standard_normal(m).astype(np.float32)
    return coo.coalesce(idx, vals)


@pytest.mark.parametrize("dims,ranks", [((4, 3, 5), (2, 3, 2)), ((5, 4, 3, 2), (2, 2, 3, 1)),
                                        ((6, 7), (3, 2))])
def test_reformulation_equals_unfolding_times_kron(dims, ranks):
    """Z_(n) = T_(n) (F_N kron ... kron F_{n+1} kron F_{n-1} kron ... kron F_1): the
    textbook identity that follows from the TTM definition and the unfolding's
    column order (Section 2.1); numpy.kron computes the right-hand side."""
    rng = np.random.default_rng(0)
    idx, vals, _ = _random_sparse(rng, dims, 40)
    F = [rng.standard_normal((L, K)) for L, K in zip(dims, ranks)]
    T = ttm.dense(idx, vals, dims)
    for n in range(len(dims)):
        kr = np.ones((1, 1))
        for j in range(len(dims)):
            if j != n:
                kr = np.kron(F[j], kr)          # later modes on the left => first remaining mode fastest
        expect = ttm.unfold(T, n) @ kr
        got = ttm.ttm_chain(idx, vals, F, n, dims)
        np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12)


def test_unfold_column_order_matches_section_2_1():
    dims = (2, 3, 4)
    T = np.arange(24, dtype=float).reshape(dims)
    U1 = ttm.unfold(T, 1)
    for l0 in range(2):
        for l1 in range(3):
            for l2 in range(4):
                assert U1[l1, l0 + 2 * l2] == T[l0, l1, l2]


def test_chain_is_commutative_and_matches_successive_ttms():
    rng = np.random.default_rng(1)
    dims, ranks = (5, 4, 6), (2, 3, 2)
    idx, vals, _ = _random_sparse(rng, dims, 60)
    F = [rng.standard_normal((L, K)) for L, K in zip(dims, ranks)]
    T = ttm.dense(idx, vals, dims)
    for n in range(3):
        others = [j for j in range(3) if j != n]
        Z1 = T
        for j in others:
            Z1 = ttm.ttm(Z1, F[j].T, j)
        Z2 = T
        for j in reversed(others):
            Z2 = ttm.ttm(Z2, F[j].T, j)
        np.testing.assert_allclose(Z1, Z2, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(ttm.unfold(Z1, n), ttm.ttm_chain(idx, vals, F, n, dims),
                                   rtol=1e-12, atol=1e-12)


def test_identity_factors_give_the_unfolding():
    rng = np.random.default_rng(2)
    dims = (3, 4, 5)
    idx, vals, _ = _random_sparse(rng, dims, 30)
    F = [np.eye(L) for L in dims]
    T = ttm.dense(idx, vals, dims)
    for n in range(3):
        np.testing.assert_array_equal(ttm.ttm_chain(idx, vals, F, n, dims), ttm.unfold(T, n))


def test_rows_subset_matches_full():
    rng = np.random.default_rng(3)
    dims, ranks = (30, 20, 10), (3, 4, 2)
    idx, vals, _ = _random_sparse(rng, dims, 500)
    F = [rng.standard_normal((L, K)) for L, K in zip(dims, ranks)]
    for n in range(3):
        full = ttm.ttm_chain(idx, vals, F, n, dims)
        pick = np.array([7, 3, 0, dims[n] - 1])
        np.testing.assert_allclose(ttm.ttm_chain_rows(idx, vals, F, n, pick), full[pick], rtol=1e-13)


def test_coalesce_brute_force():
    rng = np.random.default_rng(4)
    for trial in range(20):
        dims = (rng.integers(1, 6), rng.integers(1, 6), rng.integers(1, 4))
        m = int(rng.integers(0, 60))
        idx = [rng.integers(0, L, m) for L in dims]
        vals = rng.standard_normal(m).astype(np.float32)
        d = {}
        for e in range(m):
            key = tuple(int(i[e]) for i in idx)
            d[key] = d.get(key, 0.0) + float(vals[e])
        keys = sorted(d)
        ic, vc, nsq = coo.coalesce(idx, vals)
        ic2, vc2, nsq2 = coo.coalesce_fast(idx, vals)
        assert [tuple(int(i[k]) for i in ic) for k in range(len(vc))] == keys
        np.testing.assert_array_equal(vc, np.array([d[k] for k in keys], np.float32))
        for a, b in zip(ic, ic2):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(vc, vc2)
        assert nsq == pytest.approx(sum(float(np.float32(d[k])) ** 2 for k in keys), rel=1e-15, abs=0)
        assert nsq == nsq2


# ---- the C++/OpenMP oracle (oracle/ttm_cpp.py) --------------------------------------------------

@pytest.mark.parametrize("dims,ranks", [((4, 3, 5), (2, 3, 2)), ((5, 4, 3, 2), (2, 2, 3, 1)),
                                        ((6, 7), (3, 2)), ((3, 4, 2, 3, 2), (2, 1, 2, 3, 2))])
def test_cpp_oracle_equals_unfolding_times_kron(dims, ranks):
    """The multi-threaded FP64 TTM-chain against the dense identity
    Z_(n) = T_(n) (F_N kron ... kron F_1 without F_n), numpy.kron on the right."""
    from oracle import cpp as ttm_cpp
    rng = np.random.default_rng(3)
    idx, vals, _ = _random_sparse(rng, dims, 50)
    F = [rng.standard_normal((L, K)) for L, K in zip(dims, ranks)]
    T = ttm.dense(idx, vals, dims)
    for n in range(len(dims)):
        kr = np.ones((1, 1))
        for j in range(len(dims)):
            if j != n:
                kr = np.kron(F[j], kr)
        expect = ttm.unfold(T, n) @ kr
        np.testing.assert_allclose(ttm_cpp.ttm_chain(idx, vals, F, n, dims), expect, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["c1", "zipf"])
def test_cpp_oracle_matches_numpy_oracle(name):
    """On the c1 workload and a Zipf tensor with repeated coordinates: the full
    Z_(n), and rows of chosen slices streamed in uneven batches (including an
    empty one), equal the NumPy oracle's."""
    import synth
    from oracle import cpp as ttm_cpp
    if name == "c1":
        w = synth.make_workload("c1")
        dims, idx, vals, F = w["dims"], w["idx"], w["vals"], w["F0"]
    else:
        dims = (900, 600, 300)
        idx, vals = synth.make_tensor(dims, 80_000, "zipf", (1.2, 1.0, 1.4), "lognormal", seed=9)
        F = synth.orthonormal_init(19, dims, (7, 5, 6))
    for n in range(3):
        Zo = ttm.ttm_chain(idx, vals, F, n, dims)
        np.testing.assert_allclose(ttm_cpp.ttm_chain(idx, vals, F, n, dims), Zo, rtol=1e-12, atol=1e-12)
        pick = np.unique(np.concatenate([np.argsort(np.bincount(idx[n], minlength=dims[n]))[-5:], [0, dims[n] - 1]]))
        acc = ttm_cpp.RowAccumulator(F, n, dims[n], pick)
        m = len(vals)
        for a, b in [(0, m // 3), (m // 3, m // 3), (m // 3, m - 7), (m - 7, m)]:
            acc.add([i[a:b] for i in idx], vals[a:b])
        np.testing.assert_allclose(acc.rows, Zo[pick], rtol=1e-12, atol=1e-12)
