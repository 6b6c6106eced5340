"""Pins of the coalescing oracle at scale (oracle/coo_omp.cpp through
oracle.cpp): merged slice cardinalities and merged values against the plain
NumPy coalescing (oracle/coo.py), which is pinned by brute force elsewhere."""
import numpy as np
import pytest

from oracle import coo, cpp


def _draws(dims, m, seed):
    rng = np.random.default_rng(seed)
    # a skewed draw so coordinates repeat
    idx = [np.minimum((rng.zipf(1.6, m) - 1) % L, L - 1).astype(np.int32) for L in dims]
    return idx, rng.lognormal(0.0, 1.0, m).astype(np.float32)


@pytest.mark.parametrize("dims", [(37, 50, 11), (4_000_000, 4_000_000, 2_000_001), (7, 3, 5, 2)])
def test_distinct_counter_matches_coalesce(dims):
    """Slice sizes of the merged list, fed in three uneven batches; the second
    shape needs 65 bits per key, so it is split into two parts."""
    idx, vals = _draws(dims, 30_000, 5)
    ic, vc, _ = coo.coalesce(idx, vals)
    dc = cpp.DistinctCounter(dims)
    for a, b in [(0, 1000), (1000, 1000), (1000, 30_000)]:
        dc.add([i[a:b] for i in idx])
    m, counts = dc.finish()
    assert m == len(vc)
    for n, L in enumerate(dims):
        np.testing.assert_array_equal(counts[n], np.bincount(ic[n], minlength=L))


def test_keysums_match_coalesce():
    dims = (40, 30, 20)
    idx, vals = _draws(dims, 50_000, 6)
    ic, vc, _ = coo.coalesce(idx, vals)
    pick = np.array([0, 1, 2, 17, len(vc) // 2, len(vc) - 1])
    ks = cpp.KeySums([i[pick] for i in ic], dims[0])
    for a, b in [(0, 7), (7, 20_000), (20_000, 50_000)]:
        ks.add([i[a:b] for i in idx], vals[a:b])
    out, cnt = ks.finish()
    np.testing.assert_array_equal(out, vc[pick])
    keys = [tuple(int(i[k]) for i in ic) for k in pick]
    allk = list(zip(*[i.tolist() for i in idx]))
    assert cnt.tolist() == [sum(1 for t in allk if t == k) for k in keys]
