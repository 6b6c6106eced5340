"""Parity at the benchmark workload's full size, in the configuration the
benchmark times (default options): c2, 1,000,000 x 500,000 x 200,000, 1e8
Zipf(1.1) draws, ranks 10.

The oracle cannot run the whole workload in seconds, so it checks sampled
outputs it can compute one by one, from the drawn input (never from the
library's outputs):
  * merged values of sampled coordinates (bit-exact) and the merged key set;
  * the Lite partition of every mode (bit-exact, from the slice sizes);
  * rows of Y_(n) for sampled slices (heaviest, split over bins, random);
and properties that hold at any size for HOOI (orthonormal factors,
non-decreasing fit, determinism, BF16-Gram run ending at the FP32 fit)."""
import numpy as np
import pytest

import synth
from oracle import cpp, lite, ttm
from tests.gpu_common import fit_noise, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2(tk):
    import torch
    w = synth.make_workload("c2")
    dims = w["dims"]
    keys = (w["idx"][0].astype(np.int64) * dims[1] + w["idx"][1]) * dims[2] + w["idx"][2]
    uk = np.unique(keys)
    ctx = tk.TuckerContext(0)
    ctx.load_coo([torch.from_numpy(i).cuda() for i in w["idx"]], torch.from_numpy(w["vals"]).cuda(), dims)
    ctx.set_ranks(w["ranks"])
    print(f"c2 loaded: {len(w['vals'])} draws, {len(uk)} distinct", flush=True)
    return w, keys, uk, ctx


def test_fullsize_coalesce(c2):
    w, keys, uk, ctx = c2
    dims = w["dims"]
    m, norm_sq = ctx.tensor_info()
    assert m == len(uk)
    ic, vc = ctx.get_coo()
    gk = (ic[0].astype(np.int64) * dims[1] + ic[1]) * dims[2] + ic[2]
    np.testing.assert_array_equal(gk, uk)          # the merged key set, in canonical order
    # merged values of sampled coordinates: FP64 sum in input order, rounded once
    rng = np.random.default_rng(2024)
    pos = np.unique(np.concatenate([rng.choice(len(uk), 3000, replace=False), [0, len(uk) - 1]]))
    sk = uk[pos]
    sel = np.flatnonzero(np.isin(keys, sk))
    acc = np.zeros(len(sk), np.float64)
    np.add.at(acc, np.searchsorted(sk, keys[sel]), w["vals"][sel].astype(np.float64))
    np.testing.assert_array_equal(vc[pos], acc.astype(np.float32))
    # ||T||^2 of the merged values (FP64; only the summation order differs)
    assert abs(norm_sq - float(np.sum(vc.astype(np.float64) ** 2))) <= 1e-12 * norm_sq


def _segments(res, P):
    """(bin, slice, length, bad) of every segment, in layout order, from a LiteResult."""
    out = []
    for p in range(P):
        for s, c in res.bin_slices[p]:
            out.append((p, s, c, 1 if len(res.pieces[s]) > 1 else 0))
    return np.array(out, np.int64).reshape(-1, 4)


def test_fullsize_partition(c2):
    w, keys, uk, ctx = c2
    dims = w["dims"]
    coords = [uk // (dims[1] * dims[2]), (uk // dims[2]) % dims[1], uk % dims[2]]
    for n in range(3):
        sizes = np.bincount(coords[n], minlength=dims[n])
        g = ctx.partition(n, elem_order=False)
        st = g["stats"]
        res = lite.lite(sizes, st["P"])
        seg = _segments(res, st["P"])
        np.testing.assert_array_equal(g["seg_bin"], seg[:, 0])
        np.testing.assert_array_equal(g["seg_slice"], seg[:, 1])
        np.testing.assert_array_equal(np.diff(g["seg_begin"]), seg[:, 2])
        np.testing.assert_array_equal(g["seg_bad"], seg[:, 3])
        for k in ("E_max", "R_sum", "R_max", "n_bad"):
            assert st[k] == res.stats[k], (n, k)
        assert st["E_max"] <= st["limit"]
        assert st["R_max"] <= -(-st["L_nonempty"] // st["P"]) + 2
        print(f"mode {n}: P={st['P']} E_max={st['E_max']} R_max={st['R_max']} bad={st['n_bad']}", flush=True)


def test_fullsize_ttm_sampled_rows(c2):
    w, keys, uk, ctx = c2
    dims = w["dims"]
    for n, F in enumerate(w["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    rng = np.random.default_rng(77)
    for n in range(3):
        Y, rows = ctx.ttm_chain(n)
        sizes = np.bincount(w["idx"][n], minlength=dims[n])
        heavy = np.argsort(sizes)[::-1][:10]
        g = ctx.partition(n, elem_order=False)
        bad = np.unique(g["seg_slice"][g["seg_bad"] == 1])
        pick = np.unique(np.concatenate([heavy, rng.choice(bad, min(200, len(bad)), replace=False),
                                         rng.choice(rows, 790, replace=False)]))
        # linear in the values, so the unmerged draws give the same rows (the
        # oracle's C++/OpenMP FP64 accumulator over every draw)
        acc = cpp.RowAccumulator(w["F0"], n, dims[n], pick)
        acc.add(w["idx"], w["vals"])
        Yo = acc.rows
        Yg = Y[np.searchsorted(rows, pick)]
        err = rel_fro(Yg, Yo)
        row_err = np.linalg.norm(Yg - Yo, axis=1) / np.maximum(np.linalg.norm(Yo, axis=1), 1e-30)
        print(f"mode {n}: {len(pick)} sampled rows, rel err {err:.2e}, worst row {row_err.max():.2e}", flush=True)
        assert err <= 1e-5
        assert row_err.max() <= 1e-4


def test_fullsize_hooi_properties(c2):
    w, keys, uk, ctx = c2

    def run(prec, iters):
        ctx.set_options(prec=prec, refine=1)
        for n, F in enumerate(w["F0"]):
            ctx.set_factor(n, np.ascontiguousarray(F))
        return ctx.hooi_iterate(iters)

    fits = run("fp32", 6)
    for a, b in zip(fits, fits[1:]):
        assert b >= a - fit_noise(a)
    for n in range(3):
        F = ctx.get_factor(n)
        np.testing.assert_allclose(F.T @ F, np.eye(w["ranks"][n]), atol=1e-12)
    _, fit = ctx.core()
    assert abs(fit - fits[-1]) <= 1e-12
    again = run("fp32", 6)
    assert again == fits                             # no atomics anywhere: bit-identical
    bf = run("bf16", 6)
    print("fits fp32", fits, "bf16-gram", bf, flush=True)
    assert abs(bf[-1] - fits[-1]) <= 1e-5
