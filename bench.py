"""Benchmark: sparse HOOI on one MI355X.

A step is one HOOI invocation over all modes (TTM-chain, fixup, Gram,
eigensolve, factor, then core and fit).  The default workload is the largest
one-GPU configuration: the 3-mode tensor 4,000,000 x 4,000,000 x 2,000,000
with 4.0e9 drawn nonzeros (Zipf 0.8 / 1.2 / 1.5 per mode, lognormal values),
ranks 10 x 10 x 10.  The draws are generated on the host in chunks and
streamed into the library (tk_load_coo_begin / _append / _end), so host
memory never holds the whole list; the timed invocations run with the
tensor resident in HBM.  Prints one JSON line.

  value      TTM-chain Gnnz/s per mode = m' / (mean over modes of the
             TTM-chain + fixup time) / 1e9, from HIP events on the library's stream
  ms/step    wall time of one FP32 HOOI invocation; the same run with the
             Gram in BF16 (last invocation FP32) is reported beside it
  roofline   the TTM-chain kernel's algorithmic bytes per launch / its average
             launch time (HIP events around each launch, on the library's
             stream), against 8 TB/s; traffic = HBM bytes per launch from the
             committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this
             workload, while the kernel source is unchanged since it was taken
  cpu_baseline  the oracle's FP64 TTM-chain (C++/OpenMP, every host thread)
             timed on a bounded prefix of the same draws

  python bench.py --summarize-profile DIR --workload W   writes the profiles/
  summaries from rocprofv3 CSV output (DIR/trace, DIR/fetch, DIR/write)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 31
# the sources of the Lite-bin TTM-chain kernels (the traffic summary is keyed to them)
TTM_SOURCES = [os.path.join(ROOT, "paper_1804_09494_amd", "csrc", f) for f in ("ttm.hip", "ttm_common.hpp")]
COPY_KERNEL = "__amd_rocclr_copyBuffer"
TTM_KERNELS = {3: "k_ttm3_mfma", 4: "k_ttm4_mfma"}
CHUNK = 1 << 27          # draws per streamed chunk (2 GiB of host buffers for 3 modes)


# the sources of the kernels whose SQ counters are summarised (TTM-chain and Gram)
SQ_SOURCES = TTM_SOURCES + [os.path.join(ROOT, "paper_1804_09494_amd", "csrc", "gram.hip")]


def sq_file(workload):
    return os.path.join(ROOT, "profiles", f"sq_counters_{workload}.json")


def committed_mfma_util(workload):
    """MfmaUtil (percent of SIMD cycles with the matrix cores busy, rocprofv3's
    derived counter) per kernel template from the committed SQ summary of this
    workload, or None when those kernels' sources changed since."""
    try:
        with open(sq_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _sha256(SQ_SOURCES):
        return None
    return {k: round(v["MfmaUtil"], 1) for k, v in t["kernels"].items() if "MfmaUtil" in v and v["MfmaUtil"] > 0}


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"ttm_{workload}_hbm_traffic.json")


def _sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic(workload):
    """HBM bytes per TTM-chain launch (per mode) from the committed counter
    summary of this workload, or None when the kernel source changed since."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _sha256(TTM_SOURCES):
        return None
    return t["hbm_bytes_per_mode"]


def _counter_rows(path):
    import csv
    rows = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            key = int(r["Dispatch_Id"])
            ent = rows.setdefault(key, {"kernel": r["Kernel_Name"], "value": 0.0})
            ent["value"] += float(r["Counter_Value"])
    return [rows[k] for k in sorted(rows)]


SQ_PASSES = {
    "sqa": "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_INSTS_VALU SQ_INSTS_LDS "
           "SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE",
    "sqb": "SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_WAIT_INST_LDS SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VALU "
           "SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU GRBM_GUI_ACTIVE MfmaUtil",
}


def _summarize_sq(d, workload, regex):
    """Per-kernel means of the SQ counter passes (sqa/, sqb/ under d) of
    `bench.py --workload <w> --steps 1 --warmup 0 --no-cpu-baseline`."""
    import csv
    import glob
    per = {}
    for name in SQ_PASSES:
        f = glob.glob(os.path.join(d, name, "*counter_collection.csv"))
        if not f:
            continue
        disp = {}
        for r in csv.DictReader(open(f[0])):
            ent = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "c": {}})
            ent["c"][r["Counter_Name"]] = ent["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        for ent in disp.values():
            k = ent["kernel"].split("(")[0].replace("void ", "")
            agg = per.setdefault(k, {})
            for c, v in ent["c"].items():
                agg.setdefault(c, []).append(v)
    if not per:
        return
    lines = [f"SQ counters per dispatch (mean over dispatches), `bench.py --workload {workload} --steps 1 --warmup 0 "
             "--no-cpu-baseline`, kernels matching " + regex]
    for name, cs in SQ_PASSES.items():
        lines.append(f"command ({name}): cd /tmp && rocprofv3 --pmc {cs} --kernel-include-regex '{regex}' "
                     f"--output-format csv -d <dir>/{name} -o run -- python3 -u <repo>/bench.py --workload {workload} "
                     "--steps 1 --warmup 0 --no-cpu-baseline")
    lines.append("")
    for k, agg in sorted(per.items()):
        m = {c: sum(v) / len(v) for c, v in agg.items()}
        n = max(len(v) for v in agg.values())
        lines.append(f"{k}  ({n} dispatches)")
        for c in sorted(m):
            lines.append(f"    {c:28s} {m[c]:.6g}")
        wc = m.get("SQ_WAVE_CYCLES")
        if wc:
            for c in ("SQ_ACTIVE_INST_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                      "SQ_WAIT_INST_LDS"):
                if c in m:
                    lines.append(f"    {c} / SQ_WAVE_CYCLES = {m[c] / wc:.3f}")
        w = m.get("SQ_WAVES")
        if w:
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_MFMA", "SQ_INSTS_VMEM_RD", "SQ_INSTS_SALU"):
                if c in m:
                    lines.append(f"    {c} per wave = {m[c] / w:.1f}")
        lines.append("")
    with open(os.path.join(ROOT, "profiles", f"sq_counters_{workload}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    means = {k: {c: sum(v) / len(v) for c, v in agg.items()} for k, agg in per.items()}
    with open(sq_file(workload), "w") as f:
        json.dump({"workload": workload, "source_sha256": _sha256(SQ_SOURCES), "kernels": means}, f, indent=1)


def summarize_profile(d, workload, kernel):
    """profiles/ summaries from rocprofv3 CSV output under d: trace/ (kernel
    trace + stats of a bench run), fetch/ and write/ (FETCH_SIZE and WRITE_SIZE
    runs of `bench.py --steps 1 --warmup 0 --no-cpu-baseline`, copy and TTM
    kernels only)."""
    import csv
    import glob
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stats = glob.glob(os.path.join(d, "trace", "*kernel_stats.csv"))
    if stats:
        rows = list(csv.DictReader(open(stats[0])))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines = [f"kernel time of `bench.py --workload {workload} --steps 10 --warmup 1 --no-cpu-baseline`, top kernels",
                 "command: cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run "
                 f"-- python3 -u <repo>/bench.py --workload {workload} --steps 10 --warmup 1 --no-cpu-baseline",
                 "", f"{'total ms':>10} {'calls':>6} {'avg us':>10}  kernel"]
        for r in rows[:25]:
            lines.append(f"{float(r['TotalDurationNs']) / 1e6:10.3f} {int(r['Calls']):6d} "
                         f"{float(r['AverageNs']) / 1e3:10.1f}  {r['Name'][:110]}")
        with open(os.path.join(out_dir, f"hooi_{workload}_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    _summarize_sq(d, workload, f"{kernel}|k_gram")
    fetch_f = glob.glob(os.path.join(d, "fetch", "*counter_collection.csv"))
    write_f = glob.glob(os.path.join(d, "write", "*counter_collection.csv"))
    if not (fetch_f and write_f):
        return
    fetch, write = _counter_rows(fetch_f[0]), _counter_rows(write_f[0])
    # calibration: the bench's 2 GiB device copies (read 2 GiB, write 2 GiB)
    big = [r for r in fetch if r["kernel"] == COPY_KERNEL and r["value"] > 1e6]
    bigw = [r for r in write if r["kernel"] == COPY_KERNEL and r["value"] > 1e6]
    copy_kib = COPY_BYTES / 1024
    f_scale = copy_kib / (sum(r["value"] for r in big) / len(big))
    w_scale = copy_kib / (sum(r["value"] for r in bigw) / len(bigw))
    tf = [r["value"] for r in fetch if kernel in r["kernel"]]
    tw = [r["value"] for r in write if kernel in r["kernel"]]
    every = [round((a * f_scale + b * w_scale) * 1024) for a, b in zip(tf, tw)]
    N = {"k_ttm3_mfma": 3, "k_ttm4_mfma": 4}.get(kernel, len(every))
    res = {"kernel": kernel, "workload": workload,
           "note": "hbm_bytes_per_mode: the first invocation's launches, modes 0..N-1 in order (FP32); "
                   "every_launch: all launches of the run in order (later invocations, BF16 tiles, the HOSVD "
                   "initialisation's Jacobi sweep and its core)",
           "source_sha256": _sha256(TTM_SOURCES),
           "fetch_kib_every_launch": tf, "write_kib_every_launch": tw, "hbm_bytes_every_launch": every,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": sum(r["value"] for r in big) / len(big),
                                "write_kib": sum(r["value"] for r in bigw) / len(bigw),
                                "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
           "hbm_bytes_per_mode": every[:N],
           "commands": [f"cd /tmp && rocprofv3 --pmc {c} --kernel-include-regex '{kernel}|copyBuffer' "
                        f"--output-format csv -d <dir>/{d_} -o run -- python3 -u <repo>/bench.py --workload {workload} "
                        "--steps 1 --warmup 0 --no-cpu-baseline" for c, d_ in (("FETCH_SIZE", "fetch"),
                                                                               ("WRITE_SIZE", "write"))]}
    with open(traffic_file(workload), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def algorithmic_bytes(m, N, R, khat, dims, ranks, n):
    """Per-launch bytes the TTM-chain must move: the mode-n copy of the tensor
    (N-1 int32 coordinates + one FP32 value per nonzero), one write of the
    compact Y_(n), one read of each other factor."""
    b = m * (4 * (N - 1) + 4) + R * khat * 4
    for j in range(N):
        if j != n:
            b += dims[j] * ranks[j] * 4
    return b


def device_copy_bandwidth(torch):
    """Device-to-device copy of 2 GiB (read + write counted): the measured
    reference next to the 8 TB/s peak, and the known-size kernel the HBM
    byte counters are scaled against."""
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del src, dst
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def cpu_baseline(stream, F, target_s=15.0):
    """The oracle's FP64 TTM-chain (C++/OpenMP on every host thread) over a
    prefix of the same draws, along every mode, grown until one pass over
    the modes runs for about target_s seconds."""
    from oracle import cpp as ttm_cpp
    N = len(stream.dims)
    n_s = 1 << 20
    while True:
        n_s = min(n_s, stream.nnz)
        idx, vals = stream.chunk(0, n_s)
        t0 = time.perf_counter()
        for n in range(N):
            ttm_cpp.ttm_chain(idx, vals, F, n, stream.dims)
        el = time.perf_counter() - t0
        if el >= target_s / 3 or n_s >= stream.nnz:
            break
        n_s = int(n_s * min(8.0, max(1.5, target_s / max(el, 1e-3))))
    return {"value": round(n_s / (el / N) / 1e9, 6), "unit": "Gnnz/s/mode", "cores": ttm_cpp.threads(),
            "kind": "oracle",
            "sample": f"FP64 C++/OpenMP TTM-chain of the oracle along each of the {N} modes over the first {n_s} "
                      f"drawn nonzeros of the same workload (duplicates not merged), {el:.1f} s for the {N} modes"}


def stream_load(ctx, stream, torch):
    """Generate the draws chunk by chunk into pinned host buffers (two sets:
    the next chunk is drawn while the current one is copied) and append them."""
    N = len(stream.dims)
    bufs = []
    for _ in range(2):
        idx = [torch.empty(CHUNK, dtype=torch.int32, pin_memory=True).numpy() for _ in range(N)]
        vals = torch.empty(CHUNK, dtype=torch.float32, pin_memory=True).numpy()
        bufs.append((idx, vals))
    ctx.load_begin(stream.dims, stream.nnz)
    starts = list(range(0, stream.nnz, CHUNK))
    gen_s = 0.0

    def gen(k):
        t = time.perf_counter()
        a = starts[k]
        n = min(CHUNK, stream.nnz - a)
        idx, vals = stream.chunk(a, n, *bufs[k % 2])
        return idx, vals, time.perf_counter() - t

    with cf.ThreadPoolExecutor(1) as ex:
        fut = ex.submit(gen, 0)
        for k in range(len(starts)):
            idx, vals, g = fut.result()
            gen_s += g
            if k + 1 < len(starts):
                fut = ex.submit(gen, k + 1)
            ctx.load_append(idx, vals)
    ctx.load_end()
    return gen_s


def run_completion(args):
    """The differentiation form at its configuration's scale: Tucker completion
    on 500,000 x 500,000 x 50,000 with 2e8 observations (Zipf 1.0 per mode),
    ranks 16.  A step is one forward (model values at every observation) and
    one adjoint (gradients of the squared loss for the core and the three
    factors).  The targets are the values of a planted rank-16 model (core
    N(0,1), factors N(0, 1/16)), formed by the library's forward, plus
    N(0, 0.01^2) noise; the timed parameters are another seeded model."""
    import torch
    import synth
    import paper_1804_09494_amd as P
    torch.cuda.set_device(0)
    dims, n_obs, ranks = (500_000, 500_000, 50_000), int(2e8 * args.scale), (16, 16, 16)
    dims = tuple(max(2, int(round(d * (args.scale if args.scale < 1 else 1)))) for d in dims)
    t = time.perf_counter()
    obs = synth.make_completion(dims, n_obs, ranks)
    idx = [torch.from_numpy(i).cuda() for i in obs["idx"]]
    ctx = P.TuckerContext(0)
    ctx.load_obs(idx, dims, ranks)
    del idx
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    Gt = torch.tensor(obs["G_true"].ravel(order="F"), dtype=torch.float32, device="cuda")
    Ft = [torch.tensor(f, dtype=torch.float32, device="cuda") for f in obs["F_true"]]
    noise = torch.from_numpy(synth.normal(4949, synth.S_NOISE, n_obs).astype(np.float32)).cuda()
    v = ctx.tucker_eval(Gt, Ft) + 0.01 * noise
    del noise
    rng = np.random.default_rng(7)
    G = torch.tensor(rng.standard_normal(int(np.prod(ranks))), dtype=torch.float32, device="cuda")
    F = [torch.tensor(rng.standard_normal((d, k)) / np.sqrt(k), dtype=torch.float32, device="cuda")
         for d, k in zip(dims, ranks)]

    def step():
        m = ctx.tucker_eval(G, F)
        g = 2.0 * (m - v)
        return ctx.tucker_adjoint(g, G, F)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = adj = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e[0].record()
        m = ctx.tucker_eval(G, F)
        e[1].record()
        ctx.tucker_adjoint(2.0 * (m - v), G, F)
        e[2].record()
        torch.cuda.synchronize()
        fwd += e[0].elapsed_time(e[1])
        adj += e[1].elapsed_time(e[2])
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    out = {"metric": "Tucker-completion forward + adjoint, observations per second", "value": round(n_obs / ms / 1e6, 3),
           "unit": "Gobs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"c4: completion on {'x'.join(str(d) for d in dims)}, {n_obs} Zipf(1.0) "
                                  f"observations, ranks 16x16x16, one forward + adjoint per step"},
           "forward_ms": round(fwd / args.steps, 3), "adjoint_ms": round(adj / args.steps, 3),
           "setup_s": round(setup_s, 2)}
    # algorithmic bytes of a step: each observation's N coordinates and one
    # value in the forward (model) and again in the adjoint (residual); the
    # core and factors read by both, their gradients written by the adjoint
    N = len(dims)
    params = sum(d * k for d, k in zip(dims, ranks)) + int(np.prod(ranks))
    step_bytes = n_obs * 2 * (4 * N + 4) + 3 * 4 * params
    step_ms = (fwd + adj) / args.steps
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                       "kernel": "forward + adjoint step, all launches (HIP events)", "bytes_per_step": step_bytes}
    print(json.dumps(out), flush=True)


def run_ablation(args):
    """Partition ablations on one GPU: the TTM-chain of c2-shaped tensors
    (1,000,000 x 500,000 x 200,000, 1e8 draws, Zipf 1.1 or 1.5 on every mode,
    ranks 10) under Lite bins with the matrix-core kernel, Lite bins with the
    vector-ALU kernel, CoarseG bins (whole slices, random order, contiguous
    blocks) with the vector-ALU kernel, and no partition (atomics).  Reports
    Section 4's metrics E_max and R_max and the kernel time per mode."""
    import torch
    import synth
    import paper_1804_09494_amd as P
    torch.cuda.set_device(0)
    dims, nnz, ranks = (1_000_000, 500_000, 200_000), int(1e8 * args.scale), (10, 10, 10)
    out = {"metric": "TTM-chain ms per mode under each partition", "config": {"dims": dims, "draws": nnz,
                                                                               "ranks": ranks}, "runs": []}
    for s in (1.1, 1.5):
        idx, vals = synth.make_tensor(dims, nnz, "zipf", (s, s, s), "lognormal", seed=1811)
        F0 = synth.orthonormal_init(9511, dims, ranks)
        idx_d = [torch.from_numpy(i).cuda() for i in idx]
        vals_d = torch.from_numpy(vals).cuda()
        for scheme, kernel in (("lite", "auto"), ("lite", "vector"), ("coarse", "vector"), ("none", "atomic")):
            ctx = P.TuckerContext(0, keep_elem_order=0, partition="coarse" if scheme == "coarse" else "lite",
                                  ttm_kernel=kernel)
            ctx.load_coo(idx_d, vals_d, dims)
            if scheme == "coarse":
                for n, L in enumerate(dims):
                    ctx.set_slice_order(n, synth.permutation(61, 700 + n, L))
            ctx.set_ranks(ranks)
            for n, F in enumerate(F0):
                ctx.set_factor(n, np.ascontiguousarray(F))
            m, _ = ctx.tensor_info()
            run = {"zipf": s, "partition": scheme, "kernel": kernel, "m": m, "modes": []}
            for n in range(3):
                R, kh = ctx.ttm_shape(n)
                Y = torch.empty((R, kh), dtype=torch.float32, device="cuda")
                ctx.ttm_chain(n, Y)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(max(1, args.steps)):
                    ctx.ttm_chain(n, Y)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / max(1, args.steps)
                st = ctx.partition_stats(n)
                run["modes"].append({"ms": round(ms, 3), "Gnnz_s": round(m / ms / 1e6, 2), "E_max": st["E_max"],
                                     "R_max": st["R_max"], "R_sum": st["R_sum"], "n_bad": st["n_bad"], "P": st["P"]})
                del Y
            print(json.dumps(run), file=sys.stderr, flush=True)
            out["runs"].append(run)
            del ctx
            torch.cuda.empty_cache()
        del idx_d, vals_d
    print(json.dumps(out), flush=True)


def run_fiber_ablation(args):
    """The fiber-factored TTM-chain against the default kernels on the
    precision form's tensor (4 modes, 2,000,000 x 1,000,000 x 100,000 x 5,000,
    5e8 draws, Zipf 0.9/1.1/1.3/0.7, ranks 10) and on a three-mode tensor with
    long fibers (2,000 x 200 x 500, 1e8 draws, Zipf 0.5 on every mode, ranks
    10: hundreds of elements share each pair of the first two coordinates):
    TTM-chain kernel time per mode."""
    import torch
    import synth
    import paper_1804_09494_amd as P
    torch.cuda.set_device(0)
    out = {"metric": "TTM-chain kernel ms per mode, default kernel vs fiber-factored", "runs": []}
    cases = [("c3", None), ("long", ((2_000, 200, 500), int(1e8 * args.scale), (0.5, 0.5, 0.5)))]
    for name, spec in cases:
        if spec is None:
            stream = synth.WorkloadStream("c3", scale=args.scale)
            dims, ranks = stream.dims, stream.ranks
            idx, vals = stream.chunk(0, stream.nnz)
        else:
            dims, nnz, z = spec
            ranks = (10,) * len(dims)
            idx, vals = synth.make_tensor(dims, nnz, "zipf", z, "lognormal", seed=3131)
        idx_d = [torch.from_numpy(np.ascontiguousarray(i)).cuda() for i in idx]
        vals_d = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
        del idx, vals
        F0 = synth.orthonormal_init(3232, dims, ranks)
        for kernel in ("auto", "fiber"):
            ctx = P.TuckerContext(0, keep_elem_order=0, ttm_kernel=kernel)
            ctx.load_coo(idx_d, vals_d, dims)
            ctx.set_ranks(ranks)
            for n, F in enumerate(F0):
                ctx.set_factor(n, np.ascontiguousarray(F))
            m, _ = ctx.tensor_info()
            run = {"tensor": name, "dims": dims, "m": m, "kernel": kernel, "ms": []}
            for n in range(len(dims)):
                R, kh = ctx.ttm_shape(n)
                Y = torch.empty((R, kh), dtype=torch.float32, device="cuda")
                ctx.ttm_chain(n, Y)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(max(1, args.steps)):
                    ctx.ttm_chain(n, Y)
                e1.record()
                torch.cuda.synchronize()
                run["ms"].append(round(e0.elapsed_time(e1) / max(1, args.steps), 3))
                del Y
            print(json.dumps(run), file=sys.stderr, flush=True)
            out["runs"].append(run)
            del ctx
            torch.cuda.empty_cache()
        del idx_d, vals_d
    print(json.dumps(out), flush=True)


def run_eig_ablation(args):
    """The SVD step's two routes on one GPU: the Gram formed (then dense or
    block Krylov on G) against matrix-free block Krylov on Y, for a
    four-mode tensor of the precision form's shape at a tenth of its size
    (200,000 x 100,000 x 10,000 x 500, 5e7 draws, Zipf 0.9/1.1/1.3/0.7,
    lognormal values) at ranks 10 (Khat = 1000) and 16 (Khat = 4096).
    Reports the HOOI invocation time, its SVD-step part and the fits."""
    import torch
    import synth
    import paper_1804_09494_amd as P
    torch.cuda.set_device(0)
    dims, nnz = (200_000, 100_000, 10_000, 500), int(5e7 * args.scale)
    idx, vals = synth.make_tensor(dims, nnz, "zipf", (0.9, 1.1, 1.3, 0.7), "lognormal", seed=2020)
    idx_d = [torch.from_numpy(i).cuda() for i in idx]
    vals_d = torch.from_numpy(vals).cuda()
    out = {"metric": "HOOI invocation ms, Gram route vs matrix-free SVD step",
           "config": {"dims": dims, "draws": nnz}, "runs": []}
    iters = max(1, args.steps)
    for K in (10, 16):
        ranks = (K,) * 4
        F0 = synth.orthonormal_init(2121, dims, ranks)
        for method in ("gram", "matfree"):
            ctx = P.TuckerContext(0, keep_elem_order=0, eig_method=method)
            ctx.load_coo(idx_d, vals_d, dims)
            ctx.set_ranks(ranks)
            for n, F in enumerate(F0):
                ctx.set_factor(n, np.ascontiguousarray(F))
            ctx.hooi_iterate(1)   # warm-up
            for n, F in enumerate(F0):
                ctx.set_factor(n, np.ascontiguousarray(F))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fits = ctx.hooi_iterate(iters)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / iters
            tm = ctx.timings()
            run = {"ranks": K, "khat": K ** 3, "method": method, "ms_per_invocation": round(ms, 3),
                   "gram_ms": round(tm.get("gram", 0.0) / iters, 3), "eig_ms": round(tm.get("eig", 0.0) / iters, 3),
                   "ttm_ms": round(sum(v for k, v in tm.items() if k.startswith("ttm[")) / iters, 3),
                   "fits": fits, "counters": ctx.counters()}
            print(json.dumps(run), file=sys.stderr, flush=True)
            out["runs"].append(run)
            del ctx
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--share", type=int, default=1, help="one GPU's share of the workload's draws (dims kept)")
    ap.add_argument("--wg-nnz", type=int, default=0, help="elements per Lite bin (0 = library default)")
    ap.add_argument("--rows-cap", type=int, default=0, help="LDS rows per Lite bin (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-profile", metavar="DIR")
    ap.add_argument("--ablation", action="store_true", help="partition ablations (Lite, CoarseG, atomics)")
    ap.add_argument("--eig-ablation", action="store_true", help="SVD step: Gram route vs matrix-free")
    ap.add_argument("--fiber-ablation", action="store_true", help="TTM-chain: default kernels vs fiber-factored")
    args = ap.parse_args()
    if args.summarize_profile:
        import synth
        N = len(synth.WORKLOADS[args.workload]["dims"])
        summarize_profile(args.summarize_profile, args.workload, TTM_KERNELS.get(N, "k_ttm_cols"))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: no figure at several GPUs is measured; "
                                   "DESIGN.md describes how the path would shard", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "c4":
        run_completion(args)
        return
    if args.ablation:
        run_ablation(args)
        return
    if args.eig_ablation:
        run_eig_ablation(args)
        return
    if args.fiber_ablation:
        run_fiber_ablation(args)
        return

    import torch
    import synth
    import paper_1804_09494_amd as P

    torch.cuda.set_device(0)
    stream = synth.WorkloadStream(args.workload, scale=args.scale, share=args.share)
    dims, ranks = stream.dims, stream.ranks
    N = len(dims)
    opts = {"keep_elem_order": 0}
    if args.wg_nnz:
        opts["wg_nnz_target"] = args.wg_nnz
    if args.rows_cap:
        opts["lds_rows_cap"] = args.rows_cap
    ctx = P.TuckerContext(0, **opts)
    print(f"# {args.workload}: dims={dims} draws={stream.nnz}, streamed in chunks of {CHUNK}", file=sys.stderr,
          flush=True)
    t = time.perf_counter()
    gen_s = stream_load(ctx, stream, torch)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t
    m, _ = ctx.tensor_info()
    print(f"# loaded: m'={m}, {load_s:.1f}s (drawing {gen_s:.1f}s of it, overlapped)", file=sys.stderr, flush=True)
    t = time.perf_counter()
    ctx.set_ranks(ranks)
    torch.cuda.synchronize()
    part_s = time.perf_counter() - t
    F0 = stream.initial_factors()
    print(f"# partition+layout {part_s:.1f}s; device memory in use {torch.cuda.mem_get_info()}", file=sys.stderr,
          flush=True)

    copy_gbs = device_copy_bandwidth(torch)
    K = args.steps

    def run(prec):
        """Warm-up invocations, then K timed invocations from the initial factors."""
        ctx.set_options(prec=prec, refine=1)
        for n, F in enumerate(F0):
            ctx.set_factor(n, np.ascontiguousarray(F))
        if args.warmup > 0:
            ctx.hooi_iterate(args.warmup)
        for n, F in enumerate(F0):
            ctx.set_factor(n, np.ascontiguousarray(F))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fits = ctx.hooi_iterate(K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / K, fits, ctx.timings()

    bf_ms, bf_fits, bf_tm = run("bf16")
    ms_per_step, fits, tm = run("fp32")
    ttm_ms = [tm[f"ttm[{n}]"] / K for n in range(N)]
    kern_ms = [tm[f"ttm_kernel[{n}]"] / K for n in range(N)]
    value = m / (np.mean(ttm_ms) * 1e-3) / 1e9
    shapes = [ctx.ttm_shape(n) for n in range(N)]
    B = [algorithmic_bytes(m, N, shapes[n][0], shapes[n][1], dims, ranks, n) for n in range(N)]
    achieved = sum(B) / (sum(kern_ms) * 1e-3) / 1e9
    mfma_path = N in (3, 4) and all(ranks[j] <= 16 for j in range(N))
    kernel = TTM_KERNELS[N] if mfma_path else "k_ttm_cols"
    traffic = committed_traffic(args.workload) if (args.share == 1 and args.scale == 1.0 and mfma_path) else None
    stats = [ctx.partition_stats(n) for n in range(N)]
    print(f"# fits fp32 {fits}", file=sys.stderr, flush=True)
    print(f"# fits bf16 {bf_fits}", file=sys.stderr, flush=True)
    print(f"# per-step ms fp32: " + ", ".join(f"{k}={v / K:.3f}" for k, v in tm.items()), file=sys.stderr, flush=True)
    print(f"# per-step ms bf16: " + ", ".join(f"{k}={v / K:.3f}" for k, v in bf_tm.items()), file=sys.stderr,
          flush=True)
    # HOSVD initialisation (Kronecker-sketched range finder, one Jacobi sweep
    # over Gaussian sketches), then one invocation from it
    sk = [torch.from_numpy(S).cuda() for S in synth.gaussian_factors(7331, dims, ranks)]
    ctx.set_options(prec="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hosvd_fit = ctx.init_hosvd(sk)
    torch.cuda.synchronize()
    hosvd_ms = (time.perf_counter() - t0) * 1e3
    del sk
    hosvd_next = ctx.hooi_iterate(1)[0]
    print(f"# HOSVD init {hosvd_ms:.1f} ms, fit {hosvd_fit:.8f}, after one invocation {hosvd_next:.8f} "
          f"(from the random init: {fits[0]:.8f})", file=sys.stderr, flush=True)
    counters = ctx.counters()
    print(f"# counters {counters}", file=sys.stderr, flush=True)
    del ctx
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(stream, F0)

    desc = {"c5": "Zipf 0.8/1.2/1.5", "c2": "Zipf 1.1", "c3": "Zipf 0.9/1.1/1.3/0.7"}.get(args.workload, "Zipf")
    out = {
        "metric": "TTM-chain Gnnz/s/mode + HOOI iter time; FP32 vs BF16-Gram at rel err <=1e-5",
        "value": round(value, 3),
        "unit": "Gnnz/s/mode",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}{'/' + str(args.share) if args.share > 1 else ''}: "
                               f"{N}-mode {'x'.join(str(d) for d in dims)}, {stream.nnz} {desc} draws "
                               f"({m} after merging), lognormal values, ranks {'x'.join(str(k) for k in ranks)}, "
                               f"one HOOI invocation per step",
                   "m_coalesced": m, "draws": stream.nnz, "ranks": list(ranks)},
        "hooi_iter_ms": {"fp32": round(ms_per_step, 4), "bf16_gram": round(bf_ms, 4)},
        "bf16_gram_run": f"{K - 1} invocations with BF16 Kronecker tiles and Gram operands, then one refining FP32 invocation",
        "final_fit": {"fp32": fits[-1] if fits else None, "bf16_gram": bf_fits[-1] if bf_fits else None},
        "step_ms_bf16_gram": {k: round(v / K, 4) for k, v in bf_tm.items()},
        "ttm_ms_per_mode": [round(x, 4) for x in ttm_ms],
        "ttm_kernel_ms_per_mode": [round(x, 4) for x in kern_ms],
        "step_ms": {k: round(v / K, 4) for k, v in tm.items()},
        "hosvd_init": {"ms": round(hosvd_ms, 3), "fit": hosvd_fit, "fit_after_one_invocation": hosvd_next,
                       "random_init_fit_after_one_invocation": fits[0] if fits else None},
        "load_s": round(load_s, 2),
        "partition_s": round(part_s, 3),
        "partition_stats": stats,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(float(np.mean(traffic))) if traffic else None,
                     "traffic_bytes_per_mode": traffic,
                     "kernel": f"{kernel} (TTM-chain)",
                     "bytes_per_launch": [int(b) for b in B],
                     "mfma_util_pct": committed_mfma_util(args.workload) if args.share == 1 and args.scale == 1.0
                     else None},
        "device_copy_GBps": round(copy_gbs, 1),
        "counters": counters,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
