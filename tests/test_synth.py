"""The seeded generator: determinism, ranges and distribution sanity."""
import os
import subprocess
import sys

import numpy as np

import synth


def test_counter_mode_is_thread_count_independent():
    code = ("import synth, hashlib; i,v = synth.make_tensor((1000,500,200), 200000, 'zipf', (1.1,1.2,0.9)); "
            "print(hashlib.sha1(b''.join(x.tobytes() for x in i) + v.tobytes()).hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = set()
    for th in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=th, PYTHONPATH=root)
        outs.add(subprocess.check_output([sys.executable, "-c", code], env=env, cwd=root).strip())
    assert len(outs) == 1


def test_ranges_and_permutation():
    p = synth.permutation(3, 7, 1000)
    assert np.array_equal(np.sort(p), np.arange(1000))
    ix = synth.uniform_idx(1, 2, 37, 10000)
    assert ix.min() >= 0 and ix.max() < 37
    z = synth.zipf_idx(1, 2, 1.1, 500, 10000)
    assert z.min() >= 0 and z.max() < 500
    u = synth.u01(5, 5, 10000)
    assert u.min() >= 0 and u.max() < 1


def test_zipf_head_frequency():
    L, s, n = 1000, 1.1, 400_000
    perm = np.arange(L, dtype=np.int32)
    z = synth.zipf_idx(9, 1, s, L, n, perm=perm)
    H = np.sum(np.arange(1, L + 1, dtype=float) ** -s)
    for k in (1, 2, 10):
        expect = n * k ** -s / H
        got = np.sum(z == k - 1)
        assert abs(got - expect) < 5 * np.sqrt(expect)


def test_lognormal_moments():
    v = synth.lognormal_f32(1, 1, 200_000).astype(np.float64)
    lv = np.log(v)
    assert abs(lv.mean()) < 0.01 and abs(lv.std() - 1) < 0.01


def test_guided_zipf_equals_plain_search():
    """The guide table only narrows the search: every draw is the plain
    inverse-CDF binary search's answer, whatever the exponent and range."""
    for s, L in [(1.1, 1000), (0.8, 4_000_000), (1.5, 2_000_000), (1.2, 37), (0.7, 1)]:
        a = synth.zipf_idx_plain(1809, 3, s, L, 300_000)
        zs = synth.ZipfSampler(1809, 3, s, L)
        np.testing.assert_array_equal(zs.draw(0, 300_000), a)
        np.testing.assert_array_equal(np.concatenate([zs.draw(0, 123_457), zs.draw(123_457, 176_543)]), a)


def test_workload_stream_chunks_equal_whole_draws():
    w = synth.make_workload("c2", scale=0.001)
    st = synth.WorkloadStream("c2", scale=0.001)
    assert st.dims == w["dims"] and st.nnz == len(w["vals"]) and st.ranks == w["ranks"]
    parts = [st.chunk(a, min(30_000, st.nnz - a)) for a in range(0, st.nnz, 30_000)]
    for n in range(3):
        np.testing.assert_array_equal(np.concatenate([p[0][n] for p in parts]), w["idx"][n])
    np.testing.assert_array_equal(np.concatenate([p[1] for p in parts]), w["vals"])
    for a, b in zip(st.initial_factors(), w["F0"]):
        np.testing.assert_array_equal(a, b)
