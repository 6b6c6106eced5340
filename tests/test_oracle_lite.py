"""Pins of the Lite oracle: the paper's worked example, the metric example,
Theorem 6.1's bounds and the lemmas behind them (Section 6)."""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import lite


def test_fig_bins_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "lite_fig_bins.json")))
    pr, dv = g["printed"], g["derived_by_hand_from_the_pseudocode"]
    sizes = pr["sorted_sizes"]                 # slice ids 0..9 already in sorted order
    r = lite.lite(sizes, pr["P"])
    assert r.limit == pr["limit"]
    assert r.m == pr["m"]
    assert r.n_stage1 == pr["n_stage1"]
    # the eighth slice would land on bin 2 (round robin) and give it 23 > limit
    assert 7 % pr["P"] == 2
    loads_after_stage1 = [0] * pr["P"]
    for t in range(r.n_stage1):
        loads_after_stage1[t % pr["P"]] += sizes[t]
    assert loads_after_stage1[2] + sizes[7] == pr["load_of_bin2_if_eighth_slice_added"]
    # slice 9 (1-based) = id 8: head bin 1, tail bins 2 and 3
    bins9 = [p for p, c in r.pieces[8]]
    assert bins9[0] == pr["slice9_head_bin"] and bins9[1:] == pr["slice9_tail_bins"]
    # hand-derived counts
    for k, v in dv["pieces"].items():
        assert [list(x) for x in r.pieces[int(k) - 1]] == v
    assert [r.pieces[t][0][0] for t in range(7)] == dv["stage1_bins"]
    assert r.load == dv["loads"]
    assert r.stats["R_per_bin"] == dv["R_per_bin"]
    assert r.stats["R_sum"] == dv["R_sum"] and r.stats["R_max"] == dv["R_max"]
    assert r.stats["n_bad"] == dv["n_bad"]
    # Theorem 6.1 at this instance: R_max = ceil(10/5) + 2 is attained
    assert r.stats["R_max"] == -(-10 // 5) + 2


def test_framework_example_metrics(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "framework_example.json")))
    slice_of = {}
    for s, elems in g["slices_mode1"].items():
        for e in elems:
            slice_of[e] = int(s)
    owner = {}
    for p, elems in g["policy"].items():
        for e in elems:
            owner[e] = int(p)
    es = sorted(slice_of)
    m = lite.metrics_from_policy([slice_of[e] for e in es], [owner[e] for e in es], 3)
    assert m["R_per_bin"] == g["R_per_processor"]
    assert m["R_sum"] == g["R_sum"]
    # Lite on the same slices (sizes 3, 2, 3; P = 3; limit 3): every slice whole
    r = lite.lite([3, 2, 3], 3)
    assert r.stats["R_sum"] == g["L1"] and r.stats["n_bad"] == 0


def _check_theorem(sizes, P):
    r = lite.lite(sizes, P)
    m = sum(sizes)
    Lnz = sum(1 for s in sizes if s > 0)
    st_ = r.stats
    # Theorem 6.1 (with empty slices left out, L_n -> L_nonempty)
    assert st_["E_max"] <= -(-m // P)
    assert st_["R_sum"] <= Lnz + P
    assert st_["R_max"] <= -(-Lnz // P) + 2
    assert st_["n_bad"] <= P
    # every element placed exactly once
    for s, pcs in r.pieces.items():
        assert sum(c for _, c in pcs) == sizes[s]
        bins = [p for p, _ in pcs]
        # a bad slice sits on contiguous bins (proof of part 2); the walk skips
        # only bins that stage 1 already filled to the limit (gap 0)
        for p in range(bins[0], bins[-1] + 1):
            if p not in bins:
                assert r.load[p] == r.limit
                assert all(len(r.pieces[x]) == 1 for x, _ in r.bin_slices[p])
        assert bins == sorted(bins)
    assert set(r.pieces) == {l for l in range(len(sizes)) if sizes[l] > 0}
    # stage-1 slices are whole (good); stage-2 slices are all split (no "ugly" slice)
    for t, s in enumerate(r.order):
        if t < r.n_stage1:
            assert len(r.pieces[s]) == 1
        else:
            assert len(r.pieces[s]) >= 2
    # Lemma: the stage-1 receiver is always a least-loaded bin, loads cyclically ascending
    load = [0] * P
    for t in range(r.n_stage1):
        s = r.order[t]
        p = r.pieces[s][0][0]
        assert p == t % P
        assert load[p] == min(load)
        load[p] += sizes[s]
    return r


@settings(max_examples=300, deadline=None)
@given(st.lists(st.integers(min_value=0, max_value=60), min_size=1, max_size=80),
       st.integers(min_value=1, max_value=40))
def test_theorem_bounds_random(sizes, P):
    if sum(sizes) == 0:
        return
    _check_theorem(sizes, P)


@pytest.mark.parametrize("sizes,P", [
    ([7] * 50, 7),                 # all equal
    ([1] * 30 + [10_000], 16),     # one giant slice
    ([3, 1, 4, 1, 5], 50),         # more bins than slices
    ([1, 1, 1], 8),                # m < P (limit 1)
    ([0, 0, 9, 0], 3),             # empty slices around one slice
    ([2] * 10 + [100, 90, 80], 4),
])
def test_theorem_bounds_degenerate(sizes, P):
    _check_theorem(sizes, P)


def test_zipf_like_sizes_large():
    rng = np.random.default_rng(5)
    sizes = np.bincount(np.minimum(rng.zipf(1.3, 200_000), 5000) - 1, minlength=5000).tolist()
    for P in (1, 3, 64, 1000, 7919):
        _check_theorem(sizes, P)


def test_partition_layout_properties():
    rng = np.random.default_rng(11)
    L, m, P = 300, 5000, 37
    idx_n = np.minimum(rng.zipf(1.2, m), L) - 1
    part = lite.partition_mode(idx_n, L, P)
    assert np.array_equal(np.sort(part.elem_order), np.arange(m))
    assert part.bin_ptr[0] == 0 and part.bin_ptr[-1] == m
    assert np.all(np.diff(part.bin_ptr) <= part.stats["limit"])
    for b, s, a, e, bad in zip(part.seg_bin, part.seg_slice, part.seg_begin, part.seg_end, part.seg_bad):
        assert part.bin_ptr[b] <= a < e <= part.bin_ptr[b + 1]
        els = part.elem_order[a:e]
        assert np.all(idx_n[els] == s)
        assert np.all(np.diff(els) > 0)          # canonical order inside a piece
    # pieces of one slice are consecutive runs of its canonical element list
    for s in np.unique(part.seg_slice):
        segs = np.flatnonzero(part.seg_slice == s)
        els = np.concatenate([part.elem_order[part.seg_begin[k]:part.seg_end[k]] for k in segs])
        assert np.array_equal(els, np.flatnonzero(idx_n == s))
        assert (part.seg_bad[segs] == (1 if len(segs) > 1 else 0)).all()
    # segments tile the layout
    assert np.array_equal(part.seg_begin[1:], part.seg_end[:-1])


def test_choose_bins_bounds_rows():
    for m, Lnz, wg, cap in [(10**6, 10**5, 4096, 40), (10**4, 10**4, 4096, 10), (5, 5, 4096, 3)]:
        P = lite.choose_bins(m, Lnz, wg, cap)
        assert -(-Lnz // P) + 2 <= cap
        assert -(-m // P) <= wg or P >= -(-m // wg)


# ---- the C++ Lite (oracle/lite_seq.cpp) ---------------------------------------------------------

def _cpp_equals_python(sizes, P):
    from oracle import cpp
    res = lite.lite(sizes, P)
    st, sb, ss, sc, bad = cpp.lite(np.asarray(sizes, np.int64), P)
    segs = [(p, s, c, 1 if len(res.pieces[s]) > 1 else 0) for p in range(P) for s, c in res.bin_slices[p]]
    segs = np.array(segs, np.int64).reshape(-1, 4)
    np.testing.assert_array_equal(sb, segs[:, 0])
    np.testing.assert_array_equal(ss, segs[:, 1])
    np.testing.assert_array_equal(sc, segs[:, 2])
    np.testing.assert_array_equal(bad, segs[:, 3])
    for k in ("P", "limit", "m", "L_nonempty", "n_stage1", "E_max", "R_sum", "R_max", "n_bad"):
        assert st[k] == res.stats[k], k


def test_cpp_lite_worked_example(golden_dir):
    """The figure's ten slices over five bins, as in the Python oracle."""
    import json
    g = json.load(open(os.path.join(golden_dir, "lite_fig_bins.json")))
    _cpp_equals_python(g["printed"]["sorted_sizes"], g["printed"]["P"])
    from oracle import cpp
    st, *_ = cpp.lite(np.asarray(g["printed"]["sorted_sizes"], np.int64), g["printed"]["P"])
    dv = g["derived_by_hand_from_the_pseudocode"]
    assert st["R_sum"] == dv["R_sum"] and st["R_max"] == dv["R_max"] and st["n_bad"] == dv["n_bad"]


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(min_value=0, max_value=60), min_size=1, max_size=80),
       st.integers(min_value=1, max_value=40))
def test_cpp_lite_equals_python_random(sizes, P):
    _cpp_equals_python(sizes, P)


@pytest.mark.parametrize("sizes,P", [([0, 0, 0], 3), ([100], 7), ([1] * 50, 64), ([5, 0, 5, 0, 5], 1),
                                     ([1, 2, 3, 1000, 4, 5], 13)])
def test_cpp_lite_equals_python_degenerate(sizes, P):
    _cpp_equals_python(sizes, P)


def test_cpp_lite_zipf_sizes():
    rng = np.random.default_rng(4)
    sizes = (rng.zipf(1.3, 20_000) % 5000).tolist()
    _cpp_equals_python(sizes, 997)


# ---- CoarseG (Section 5) ----------------------------------------------------------------------

def test_coarse_g_hand_example():
    """Sizes 5,1,3,1 (m = 10) in the order 2,0,3,1 over P = 3 bins: prefixes
    0, 3, 8, 9 give bins floor(0*3/10)=0, floor(9/10)=0, floor(24/10)=2,
    floor(27/10)=2; bin 1 stays empty although bin 0 holds 8 elements."""
    r = lite.coarse_g([5, 1, 3, 1], 3, [2, 0, 3, 1])
    assert r.bin_slices == [[(2, 3), (0, 5)], [], [(3, 1), (1, 1)]]
    assert r.load == [8, 0, 2]
    assert r.stats["E_max"] == 8 and r.stats["R_sum"] == 4 and r.stats["R_max"] == 2 and r.stats["n_bad"] == 0


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(min_value=0, max_value=60), min_size=1, max_size=80),
       st.integers(min_value=1, max_value=40), st.randoms(use_true_random=False))
def test_coarse_g_properties(sizes, P, rnd):
    """Every slice whole in one bin (no bad slices, R_sum = L_nonempty, the
    optimum the paper states for coarse grained schemes), blocks contiguous
    in the given order, every element placed."""
    order = list(range(len(sizes)))
    rnd.shuffle(order)
    r = lite.coarse_g(sizes, P, order)
    nz = [l for l in order if sizes[l] > 0]
    assert r.stats["n_bad"] == 0
    assert r.stats["R_sum"] == len(nz)
    assert sum(r.load) == sum(sizes)
    flat = [s for b in r.bin_slices for s, _ in b]
    assert flat == nz                                   # bins in order hold the slices in the given order
    bins = [r.pieces[l][0][0] for l in nz]
    assert bins == sorted(bins)
