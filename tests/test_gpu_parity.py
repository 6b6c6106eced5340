"""GPU parity against the FP64 oracle, through the C ABI.

Bit-exact: coalescing (coordinates and merged values), the Lite partition
(bin offsets, element order, segments, statistics).  Tolerance: Y_(n), factors,
core and fit (relative Frobenius 1e-5 for the FP32 path)."""
import numpy as np
import pytest

import synth
from oracle import coo, hooi, lite, ttm
from tests.gpu_common import (U32, completion_targets, factor_tolerance, fit_noise, oracle_Y, rel_fro,
                              uniform_tensor, zipf_tensor)

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _load(P, idx, vals, dims, ranks=None, **opt):
    ctx = P.TuckerContext(0, **opt)
    ctx.load_coo([np.ascontiguousarray(i, np.int32) for i in idx], np.ascontiguousarray(vals, np.float32), dims)
    if ranks is not None:
        ctx.set_ranks(ranks)
    return ctx


# ---- coalescing ---------------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["dups", "c1", "single", "empty"])
def test_coalesce_bit_exact(tk, case):
    rng = np.random.default_rng(5)
    if case == "dups":
        dims = (7, 5, 3)
        idx = [rng.integers(0, L, 3000).astype(np.int32) for L in dims]
        vals = rng.standard_normal(3000).astype(np.float32)
    elif case == "c1":
        w = synth.make_workload("c1")
        dims, idx, vals = w["dims"], w["idx"], w["vals"]
    elif case == "single":
        dims, idx, vals = (3, 4), [np.array([2], np.int32), np.array([1], np.int32)], np.array([1.5], np.float32)
    else:
        dims, idx, vals = (3, 4, 5), [np.zeros(0, np.int32)] * 3, np.zeros(0, np.float32)
    print("case", case, dims, len(vals), flush=True)
    ctx = _load(tk, idx, vals, dims)
    m, nsq = ctx.tensor_info()
    ic, vc, nsq_o = coo.coalesce_fast(idx, vals)
    assert m == len(vc)
    gi, gv = ctx.get_coo()
    for a, b in zip(gi, ic):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(gv, vc)
    assert nsq == pytest.approx(nsq_o, rel=1e-12, abs=0)


def test_invalid_coordinates_rejected(tk):
    import paper_1804_09494_amd as P
    ctx = P.TuckerContext(0)
    idx = [np.array([0, 5], np.int32), np.array([0, 1], np.int32)]
    with pytest.raises(P.TuckerError, match="INVALID_ARG"):
        ctx.load_coo(idx, np.array([1, 2], np.float32), (5, 3))
    with pytest.raises(P.TuckerError, match="INVALID_ARG"):
        ctx.load_coo([np.array([0], np.int32)] * 2, np.array([np.nan], np.float32), (5, 3))
    with pytest.raises(P.TuckerError, match="STATE"):
        ctx.hooi_iterate(1)


# ---- Lite partition -----------------------------------------------------------------------------

PART_CASES = {
    "c1_wg64": (lambda: uniform_tensor((200, 150, 100), 20_000, seed=1805), 64),
    "zipf_wg256": (lambda: zipf_tensor((3000, 2000, 500), 60_000, s=1.3, seed=21), 256),
    "zipf_wg4096": (lambda: zipf_tensor((30_000, 20_000, 5_000), 400_000, s=1.1, seed=22), 4096),
    "giant_slice": (lambda: ([np.concatenate([np.zeros(5000, np.int32), np.arange(300, dtype=np.int32)]),
                              np.arange(5300, dtype=np.int32) % 97, np.arange(5300, dtype=np.int32) % 13],
                             np.ones(5300, np.float32)), 128),
    "tiny": (lambda: ([np.array([0, 1, 1], np.int32), np.array([2, 0, 1], np.int32),
                       np.array([0, 0, 0], np.int32)], np.array([1, 2, 3], np.float32)), 4096),
    "4mode": (lambda: zipf_tensor((500, 400, 300, 50), 30_000, s=(0.9, 1.1, 1.3, 0.7), seed=23), 512),
}


@pytest.mark.parametrize("name", list(PART_CASES))
def test_partition_bit_exact(tk, name):
    make, wg = PART_CASES[name]
    idx, vals = make()
    dims = tuple(int(max(i.max(), 0)) + 1 for i in idx)
    if name.startswith("c1"):
        dims = (200, 150, 100)
    ranks = tuple(min(3, d) for d in dims)
    print("case", name, dims, len(vals), "wg", wg, flush=True)
    ctx = _load(tk, idx, vals, dims, ranks, wg_nnz_target=wg)
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    m = len(vc)
    for n in range(len(dims)):
        g = ctx.partition(n)
        st = g["stats"]
        P = st["P"]
        assert P >= -(-m // wg)
        o = lite.partition_mode(ic[n], dims[n], P)
        np.testing.assert_array_equal(g["bin_ptr"], o.bin_ptr)
        np.testing.assert_array_equal(g["elem_order"], o.elem_order)
        np.testing.assert_array_equal(g["seg_bin"], o.seg_bin)
        np.testing.assert_array_equal(g["seg_slice"], o.seg_slice)
        np.testing.assert_array_equal(g["seg_begin"][:-1], o.seg_begin)
        assert g["seg_begin"][-1] == m
        np.testing.assert_array_equal(g["seg_bad"], o.seg_bad)
        for k in ("P", "limit", "m", "L_nonempty", "n_stage1", "E_max", "R_sum", "R_max", "n_bad"):
            assert st[k] == o.stats[k], k
        # Theorem 6.1 on the GPU's own output
        assert st["E_max"] <= st["limit"]
        assert st["R_sum"] <= st["L_nonempty"] + P
        assert st["R_max"] <= -(-st["L_nonempty"] // P) + 2


# ---- TTM-chain ----------------------------------------------------------------------------------

TTM_CASES = {
    "c1_k5": (lambda: uniform_tensor((200, 150, 100), 20_000, seed=1805), (5, 5, 5), 4096),
    "zipf_k10": (lambda: zipf_tensor((5000, 3000, 800), 200_000, s=1.1, seed=31), (10, 10, 10), 4096),
    "zipf_k10_smallbins": (lambda: zipf_tensor((5000, 3000, 800), 200_000, s=1.5, seed=32), (10, 10, 10), 300),
    "k16": (lambda: zipf_tensor((900, 700, 300), 50_000, s=1.0, seed=33), (16, 16, 16), 2048),
    "odd_ranks": (lambda: zipf_tensor((400, 300, 200), 30_000, s=1.2, seed=34), (2, 3, 7), 1024),
    "4mode_k10": (lambda: zipf_tensor((600, 500, 200, 40), 40_000, s=(0.9, 1.1, 1.3, 0.7), seed=35),
                  (10, 10, 10, 10), 2048),
    "4mode_odd": (lambda: zipf_tensor((300, 200, 100, 30), 20_000, s=1.0, seed=36), (3, 4, 2, 5), 1024),
    # K_b K_c = 256: sixteen output tiles per step in the four-mode kernel
    "4mode_k16": (lambda: zipf_tensor((300, 200, 100, 40), 20_000, s=1.0, seed=40), (4, 16, 16, 16), 1024),
    # 14 / 14 / 12 / 11 and 13 / 13 / 8 / 9 output tiles: the widths held to
    # two waves per SIMD, and the widest three-wave one
    "4mode_wide_a": (lambda: zipf_tensor((300, 200, 100, 40), 20_000, s=1.0, seed=49), (5, 12, 14, 15), 1024),
    "4mode_wide_b": (lambda: zipf_tensor((300, 200, 100, 40), 20_000, s=1.0, seed=50), (3, 9, 16, 13), 1024),
    # ranks above 16: the vector-ALU kernel (K̂ = 340, 544, 640)
    "k32_vector": (lambda: zipf_tensor((500, 400, 300), 30_000, s=1.0, seed=45), (32, 20, 17), 1024),
    # the default bin size (448 elements for the three-mode matrix-core kernel)
    "default_bins": (lambda: zipf_tensor((5000, 3000, 800), 200_000, s=1.1, seed=46), (10, 10, 10), 0),
    # four modes with a rank above 16: mode 0 on the four-mode matrix-core kernel,
    # modes 1-3 on the vector-ALU kernel with K_a = 20
    "4mode_k20": (lambda: zipf_tensor((300, 200, 100, 40), 20_000, s=1.0, seed=48), (20, 6, 5, 4), 1024),
    "2mode": (lambda: zipf_tensor((2000, 1500), 40_000, s=1.1, seed=37), (8, 6), 1024),
    "5mode": (lambda: zipf_tensor((60, 50, 40, 30, 20), 20_000, s=1.0, seed=38), (3, 2, 4, 2, 3), 512),
    # one slice split over ~19,000 bins of 16: a fixup tree of two levels (runs of 128)
    "deep_fixup": (lambda: _giant_slice_tensor(300_000, 3_000, seed=39), (4, 4, 4), 16),
}


def _giant_slice_tensor(n_giant, n_rest, seed):
    rng = np.random.default_rng(seed)
    i0 = np.concatenate([np.zeros(n_giant, np.int32), rng.integers(1, 500, n_rest, dtype=np.int32)])
    j = np.arange(n_giant + n_rest)
    i1 = (j % 3001).astype(np.int32)
    i2 = ((j * 7) % 997).astype(np.int32)
    return [i0, i1, i2], rng.standard_normal(n_giant + n_rest).astype(np.float32)


@pytest.mark.parametrize("name", list(TTM_CASES))
def test_ttm_chain_parity(tk, name):
    make, ranks, wg = TTM_CASES[name]
    idx, vals = make()
    dims = tuple(int(i.max()) + 1 for i in idx)
    print("case", name, dims, len(vals), ranks, flush=True)
    ctx = _load(tk, idx, vals, dims, ranks, wg_nnz_target=wg)
    F = [synth.normal(77, 200 + n, d * k).reshape(d, k) for n, (d, k) in enumerate(zip(dims, ranks))]
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    ic, vc, _ = coo.coalesce_fast(idx, vals)
    F32 = [f.astype(np.float32).astype(np.float64) for f in F]   # the kernel gathers FP32 factor copies
    for n in range(len(dims)):
        Y, rows = ctx.ttm_chain(n)
        Yo, rows_o = oracle_Y(ic, vc, F32, n, dims)
        np.testing.assert_array_equal(rows, rows_o)
        err = rel_fro(Y, Yo)
        print(f"  mode {n}: R={len(rows)} rel_err={err:.3e}", flush=True)
        assert err <= TOL


def test_ttm_chain_into_unaligned_device_buffer(tk):
    """The kernels store rows 16 bytes at a time.  A device Y that is not
    16-byte aligned (a view one float into its allocation) still gets the same
    rows, bit for bit, through the library's buffer; the allocation-free call
    rejects it before launching anything."""
    import torch
    idx, vals = zipf_tensor((3000, 2000, 500), 60_000, s=1.2, seed=71)
    dims = tuple(int(i.max()) + 1 for i in idx)
    ctx = _load(tk, idx, vals, dims, (10, 10, 10))
    for n, d in enumerate(dims):
        ctx.set_factor(n, synth.normal(81, 200 + n, d * 10).reshape(d, 10))
    for n in range(3):
        R, kh = ctx.ttm_shape(n)
        Ya, _ = ctx.ttm_chain(n, device=True)
        buf = torch.full((R * kh + 1,), float("nan"), dtype=torch.float32, device="cuda")
        Yu = buf[1:].view(R, kh)
        assert Yu.data_ptr() % 16 != 0
        ctx.ttm_chain(n, Yu, torch.empty(R, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yu)
        with pytest.raises(tk.TuckerError, match="INVALID_ARG"):
            ctx.ttm_chain_noalloc(n, Yu)


def test_ttm_empty_tensor(tk):
    dims = (4, 5, 6)
    ctx = _load(tk, [np.zeros(0, np.int32)] * 3, np.zeros(0, np.float32), dims, (2, 2, 2))
    for n in range(3):
        Y, rows = ctx.ttm_chain(n)
        assert Y.shape == (0, 4) and rows.shape == (0,)


DET_CASES = ["zipf_k10_smallbins", "4mode_k10", "2mode", "5mode", "k32_vector", "4mode_k20", "deep_fixup"]


@pytest.mark.parametrize("name", DET_CASES)
def test_ttm_deterministic(tk, name):
    """Reruns are bit-identical for every kernel family (three-mode and
    four-mode matrix-core kernels, the vector-ALU kernel for two, five and
    high-rank modes, and the fixup tree): no sum depends on timing."""
    make, ranks, wg = TTM_CASES[name]
    idx, vals = make()
    dims = tuple(int(i.max()) + 1 for i in idx)
    print("case", name, dims, len(vals), ranks, flush=True)
    ctx = _load(tk, idx, vals, dims, ranks, wg_nnz_target=wg)
    F = synth.orthonormal_init(5, dims, ranks)
    for n in range(len(dims)):
        ctx.set_factor(n, F[n])
    for n in range(len(dims)):
        a, _ = ctx.ttm_chain(n)
        b, _ = ctx.ttm_chain(n)
        np.testing.assert_array_equal(a, b)


# ---- HOOI ---------------------------------------------------------------------------------------

def _last_sigmas(ic, vc, dims, ranks, o, n):
    """Singular values of Z_(n) formed with the oracle's final factors: they
    qualify how well the leading K_n-subspace is determined."""
    Z = ttm.ttm_chain(ic, vc, o["factors"], n, dims)
    return np.linalg.svd(Z, compute_uv=False)


def core_tolerance(svs, ranks, tol=1e-5):
    """Allowed relative error of the sign-aligned core, or None where a
    cluster inside the leading K singular values leaves the individual
    columns (and so the core's entries) undetermined.  Each column k is
    determined to about sqrt(2) c u sigma_1^2 / min_gap_k (sin-theta theorem
    for one vector), with min_gap_k the distance of sigma_k^2 from its
    neighbours."""
    worst = tol
    for sv, K in zip(svs, ranks):
        s2 = np.asarray(sv[:K + 1], np.float64) ** 2
        for k in range(min(K, len(s2))):
            gaps = [s2[k - 1] - s2[k]] if k > 0 else []
            if k + 1 < len(s2):
                gaps.append(s2[k] - s2[k + 1])
            g = min(gaps) if gaps else s2[0]
            if g <= 1e-3 * s2[k]:
                return None
            worst = max(worst, np.sqrt(2.0) * 4.0 * U32 * s2[0] / g)
    return worst


def _hooi_compare(P, w, iters, tol_fit=1e-5, tol_proj=1e-5, sweep="gauss_seidel"):
    dims, ranks = w["dims"], w["ranks"]
    ctx = _load(P, w["idx"], w["vals"], dims, ranks, sweep=sweep)
    for n, F in enumerate(w["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    fits = ctx.hooi_iterate(iters)
    ic, vc, _ = coo.coalesce_fast(w["idx"], w["vals"])
    o = hooi.hooi(ic, vc, dims, w["F0"], ranks, iters, sweep=sweep)
    print("fits gpu", fits, "oracle", o["fits"], flush=True)
    for a, b in zip(fits, o["fits"]):
        assert abs(a - b) <= tol_fit
    svs = []
    for n in range(len(dims)):
        Fg = ctx.get_factor(n)
        np.testing.assert_allclose(Fg.T @ Fg, np.eye(ranks[n]), atol=1e-12)
        K = ranks[n]
        d = hooi.projector_distance(Fg, o["factors"][n])
        sv = _last_sigmas(ic, vc, dims, ranks, o, n)
        svs.append(sv)
        allowed, cond = factor_tolerance(sv, K, tol_proj)
        print(f"  mode {n}: projector distance {d:.3e} (allowed {allowed:.3e}, cond {cond:.3e})", flush=True)
        assert d <= allowed
    core, fit = ctx.core()
    assert abs(fit - o["fits"][-1]) <= tol_fit
    Go = o["core"]
    # rotation-invariant: the singular values of every unfolding of the core
    for n in range(len(dims)):
        sg_g = np.linalg.svd(np.moveaxis(core, n, 0).reshape(ranks[n], -1), compute_uv=False)
        sg_o = np.linalg.svd(np.moveaxis(Go, n, 0).reshape(ranks[n], -1), compute_uv=False)
        assert rel_fro(sg_g, sg_o) <= 1e-5, n
    # entrywise, up to the factors' column signs, where the columns are determined
    Fs = [ctx.get_factor(n) for n in range(len(dims))]
    sg = [np.sign(np.sum(Fs[n] * o["factors"][n], axis=0)) for n in range(len(dims))]
    Ga = core.copy()
    for n in range(len(dims)):
        shape = [1] * len(dims)
        shape[n] = ranks[n]
        Ga = Ga * sg[n].reshape(shape)
    tol_core = core_tolerance(svs, ranks)
    err_core = rel_fro(Ga, Go)
    print(f"  core: rel err {err_core:.3e} (allowed {tol_core})", flush=True)
    if tol_core is not None:
        assert err_core <= tol_core
    return ctx, fits, o


def test_hooi_c1_gauss_seidel(tk):
    w = synth.make_workload("c1")
    _hooi_compare(tk, w, 3)


def test_hooi_c1_jacobi_sweep(tk):
    w = synth.make_workload("c1")
    _hooi_compare(tk, w, 2, sweep="jacobi")


def test_hooi_zipf_small_c2_shape(tk):
    w = synth.make_workload("c2", scale=0.002)     # 2000 x 1000 x 400, 200k nonzeros, Zipf(1.1), K = 10
    _hooi_compare(tk, w, 2)


def _wide_workload(dims, nnz, zipf, ranks, seed):
    idx, vals = synth.make_tensor(dims, nnz, "zipf", zipf, "lognormal", seed=seed)
    return {"dims": dims, "ranks": ranks, "idx": idx, "vals": vals,
            "F0": synth.orthonormal_init(seed + 7690, dims, ranks)}


def test_hooi_wide_khat_block_krylov(tk):
    """Khat = 216 (4 modes, ranks 6): the eigensolve takes the block-Krylov path."""
    w = _wide_workload((300, 200, 120, 60), 40_000, (0.9, 1.1, 1.3, 0.7), (6, 6, 6, 6), 41)
    _hooi_compare(tk, w, 2)


def test_hooi_ranks_above_16(tk):
    """Ranks 20 / 18 / 17: the vector-ALU TTM-chain, the factor step without
    matrix cores, the general Cholesky and the dense eigensolve for more than
    16 pairs (K̂ = 306, 340, 360)."""
    w = _wide_workload((300, 250, 200), 40_000, (1.0, 1.1, 1.2), (20, 18, 17), 44)
    _hooi_compare(tk, w, 2)


def test_hooi_rank_one(tk):
    """Ranks 1 / 1 / 1: one-column factors, a 1 x 1 Gram, one-column rows of Y."""
    w = _wide_workload((400, 300, 200), 30_000, (1.0, 1.1, 1.2), (1, 1, 1), 47)
    _hooi_compare(tk, w, 2)


def test_hooi_full_rank_dense_reconstruction(tk):
    """K_n = L_n on a dense-filled 6 x 5 x 4 tensor: the model reproduces T, so
    the core carries all of ||T|| and every factor is square orthogonal.  The
    fit 1 - sqrt(||T||^2 - ||G||^2)/||T|| takes the square root of a rounding
    residual here, so it is held to 1e-3 while ||G|| is held to 1e-6."""
    dims = (6, 5, 4)
    g = np.indices(dims).reshape(3, -1).astype(np.int32)
    idx = [np.ascontiguousarray(g[n]) for n in range(3)]
    vals = synth.normal(91, 0, g.shape[1]).astype(np.float32)
    ctx = _load(tk, idx, vals, dims, dims)
    F0 = synth.orthonormal_init(4243, dims, dims)
    for n, F in enumerate(F0):
        ctx.set_factor(n, np.ascontiguousarray(F))
    fits = ctx.hooi_iterate(2)
    core, fit = ctx.core()
    tn = np.linalg.norm(vals.astype(np.float64))
    print("fits", fits, "||G||/||T||", np.linalg.norm(core) / tn, flush=True)
    assert abs(np.linalg.norm(core) / tn - 1.0) <= 1e-6
    assert fit >= 1.0 - 1e-3
    for n in range(3):
        Fg = ctx.get_factor(n)
        np.testing.assert_allclose(Fg.T @ Fg, np.eye(dims[n]), atol=1e-12)
        np.testing.assert_allclose(Fg @ Fg.T, np.eye(dims[n]), atol=1e-12)


def test_hooi_khat_1000_precision_form_shape(tk):
    """The precision form's shape at small scale: 4 modes, ranks 10 (Y_(n) has
    1000 columns), Zipf 0.9/1.1/1.3/0.7; FP32 path against the oracle."""
    w = _wide_workload((400, 300, 200, 60), 60_000, (0.9, 1.1, 1.3, 0.7), (10, 10, 10, 10), 42)
    _hooi_compare(tk, w, 2)


def test_hooi_fit_non_decreasing_and_timings(tk):
    w = synth.make_workload("c2", scale=0.001)
    ctx = _load(tk, w["idx"], w["vals"], w["dims"], w["ranks"])
    for n, F in enumerate(w["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    fits = ctx.hooi_iterate(4)
    for a, b in zip(fits, fits[1:]):
        assert b >= a - fit_noise(a)
    t = ctx.timings()
    assert set(t) >= {"gram", "eig", "factor", "core"}
    assert all(f"ttm[{n}]" in t and f"ttm_kernel[{n}]" in t for n in range(3))
    assert all(0 < t[f"ttm_kernel[{n}]"] <= t[f"ttm[{n}]"] for n in range(3))


def test_rank_deficient_completion(tk):
    # mode-0 has 3 nonempty slices but rank 4: the factor must be completed
    idx = [np.array([0, 1, 2, 0, 1], np.int32), np.array([0, 1, 2, 3, 4], np.int32),
           np.array([0, 0, 1, 1, 0], np.int32)]
    vals = np.array([1, 2, 3, 4, 5], np.float32)
    dims, ranks = (6, 5, 2), (4, 2, 2)
    ctx = _load(tk, idx, vals, dims, ranks)
    F0 = synth.orthonormal_init(3, dims, ranks)
    for n in range(3):
        ctx.set_factor(n, F0[n])
    ctx.hooi_iterate(1)
    F = ctx.get_factor(0)
    np.testing.assert_allclose(F.T @ F, np.eye(4), atol=1e-12)
    # the missing column is the unit vector at the lowest-index empty slice (3)
    np.testing.assert_array_equal(F[:, 3], np.eye(6)[3])
    assert np.all(F[3:, :3] == 0.0)


def test_rank_deficient_mid_sweep_matches_oracle(tk):
    # mode-0 unfolding of rank 1 with 8 nonempty slices and K_0 = 3: the failure
    # is found at the end of the invocation, mode 0 is completed and modes 1
    # and 2 run again with it.  Completed columns are orthogonal to the range of
    # T_(0), so modes 1 and 2 (and the fit) are unique and must match the oracle.
    rng = np.random.default_rng(5)
    a = rng.uniform(0.5, 1.5, 8)
    B = rng.standard_normal((6, 5))
    i0, i1, i2 = np.meshgrid(np.arange(8), np.arange(6), np.arange(5), indexing="ij")
    idx = [i0.ravel().astype(np.int32), i1.ravel().astype(np.int32), i2.ravel().astype(np.int32)]
    vals = (a[i0] * B[i1, i2]).ravel().astype(np.float32)
    dims, ranks = (8, 6, 5), (3, 2, 2)
    ctx = _load(tk, idx, vals, dims, ranks)
    F0 = synth.orthonormal_init(11, dims, ranks)
    for n in range(3):
        ctx.set_factor(n, F0[n])
    fits = ctx.hooi_iterate(2)
    o = hooi.hooi(idx, vals.astype(np.float64), dims, F0, ranks, 2)
    for n in range(3):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(ranks[n]), atol=1e-12)
    assert hooi.projector_distance(ctx.get_factor(0)[:, :1], o["factors"][0][:, :1]) <= 1e-5
    for n in (1, 2):
        assert hooi.projector_distance(ctx.get_factor(n), o["factors"][n]) <= 1e-5, n
    np.testing.assert_allclose(fits, o["fits"], atol=1e-6)


# ---- completion (differentiation form) ----------------------------------------------------------

@pytest.mark.parametrize("kernel", ["auto", "vector"])
def test_completion_eval_and_adjoint_match_oracle(tk, kernel):
    """auto: the adjoint's TTM-chains fetch the residuals through the layout
    order while staging each bin; vector: they are gathered into layout order
    by a separate pass first."""
    import torch
    from oracle import completion
    d = synth.make_completion((100, 100, 50), 20_000, (16, 16, 16), seed=4949)
    dims, ranks = d["dims"], d["ranks"]
    ctx = tk.TuckerContext(0, ttm_kernel=kernel)
    ctx.load_obs([torch.from_numpy(i).cuda() for i in d["idx"]], dims, ranks)
    rng = np.random.default_rng(1)
    G = rng.standard_normal(ranks) * 0.5
    F = [rng.standard_normal((L, K)) / np.sqrt(K) for L, K in zip(dims, ranks)]
    Gt = torch.tensor(G.ravel(order="F"), dtype=torch.float32, device="cuda")
    Ft = [torch.tensor(f, dtype=torch.float32, device="cuda") for f in F]
    G32 = Gt.double().cpu().numpy().reshape(ranks, order="F")
    F32 = [f.double().cpu().numpy() for f in Ft]
    mv = ctx.tucker_eval(Gt, Ft).double().cpu().numpy()
    mo = completion.model_values(G32, F32, d["idx"])
    assert rel_fro(mv, mo) <= TOL
    vals = completion_targets(d).astype(np.float64)
    g = 2.0 * (mo - vals)
    dG, dF = ctx.tucker_adjoint(torch.tensor(g, dtype=torch.float32, device="cuda"), Gt, Ft)
    dGo, dFo = completion.gradient(G32, F32, d["idx"], g=g.astype(np.float32).astype(np.float64))
    assert rel_fro(dG.double().cpu().numpy(), dGo.ravel(order="F")) <= TOL
    for n in range(3):
        assert rel_fro(dF[n].double().cpu().numpy(), dFo[n]) <= TOL


@pytest.mark.parametrize("dims,ranks", [((20, 300, 200), (5, 16, 7)), ((300, 15, 200), (9, 3, 12)),
                                         ((120, 90, 60), (1, 2, 1))])
def test_completion_eval_grouped_by_each_mode(tk, dims, ranks):
    """The three-mode forward walks the observations slice by slice of the mode
    with the fewest nonempty slices: each mode in turn, odd ranks."""
    import torch
    from oracle import completion
    d = synth.make_completion(dims, 15_000, ranks, seed=5151)
    ctx = tk.TuckerContext(0)
    ctx.load_obs([torch.from_numpy(i).cuda() for i in d["idx"]], dims, ranks)
    rng = np.random.default_rng(3)
    Gt = torch.tensor(rng.standard_normal(int(np.prod(ranks))), dtype=torch.float32, device="cuda")
    Ft = [torch.tensor(rng.standard_normal((L, K)) / np.sqrt(K), dtype=torch.float32, device="cuda")
          for L, K in zip(dims, ranks)]
    G32 = Gt.double().cpu().numpy().reshape(ranks, order="F")
    F32 = [f.double().cpu().numpy() for f in Ft]
    mv = ctx.tucker_eval(Gt, Ft).double().cpu().numpy()
    mo = completion.model_values(G32, F32, d["idx"])
    assert rel_fro(mv, mo) <= TOL


def test_completion_autograd_function(tk):
    import torch
    from oracle import completion
    d = synth.make_completion((40, 30, 20), 3000, (4, 3, 5), seed=17)
    ctx = tk.TuckerContext(0)
    ctx.load_obs([torch.from_numpy(i).cuda() for i in d["idx"]], d["dims"], d["ranks"])
    rng = np.random.default_rng(2)
    G = torch.tensor(rng.standard_normal(60), dtype=torch.float32, device="cuda", requires_grad=True)
    F = [torch.tensor(rng.standard_normal((L, K)), dtype=torch.float32, device="cuda", requires_grad=True)
         for L, K in zip(d["dims"], d["ranks"])]
    vals = completion_targets(d)
    v = torch.tensor(vals, device="cuda")
    m = tk.TuckerEval.apply(ctx, G, *F)
    loss = ((m - v) ** 2).sum()
    loss.backward()
    G64 = G.detach().double().cpu().numpy().reshape(d["ranks"], order="F")
    F64 = [f.detach().double().cpu().numpy() for f in F]
    dGo, dFo = completion.gradient(G64, F64, d["idx"], vals=vals)
    assert rel_fro(G.grad.double().cpu().numpy(), dGo.ravel(order="F")) <= 1e-4
    for n in range(3):
        assert rel_fro(F[n].grad.double().cpu().numpy(), dFo[n]) <= 1e-4
