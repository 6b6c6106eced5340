"""Benchmark: sparse HOOI on one MI355X.

A step is one HOOI invocation over all modes (TTM-chain, fixup, Gram,
eigensolve, factor, then core and fit) on the 3-mode Zipf(1.1) tensor
1,000,000 x 500,000 x 200,000 with 1e8 nonzeros, lognormal values, ranks
10 x 10 x 10, inputs resident in HBM.  Prints one JSON line.

  value      TTM-chain Gnnz/s per mode = m' / (mean over modes of the
             TTM-chain + fixup time) / 1e9, from HIP events on the library's stream
  ms/step    wall time of one FP32 HOOI invocation; the same run with the
             Gram in BF16 (last invocation FP32) is reported beside it
  roofline   the TTM-chain kernel's algorithmic bytes per launch / its average
             launch time, against 8 TB/s; traffic = HBM bytes per launch from
             the committed rocprofv3 counter summary, while the kernel source
             is unchanged since it was taken
  cpu_baseline  the FP64 oracle's TTM-chain timed on a bounded sample on the host

  python bench.py --summarize-profile DIR   writes the profiles/ summaries from
  rocprofv3 CSV output (DIR/trace, DIR/fetch, DIR/write; see profiles/README.md)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 31
TTM_SOURCE = os.path.join(ROOT, "paper_1804_09494_amd", "csrc", "ttm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ttm3_mfma_c2_hbm_traffic.json")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
TTM_KERNEL = "k_ttm3_mfma"


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def committed_traffic():
    """HBM bytes per TTM-chain launch (per mode) from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _sha256(TTM_SOURCE):
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


def summarize_profile(d):
    """profiles/ summaries from rocprofv3 CSV output under d: trace/ (kernel
    trace + stats of a bench run), fetch/ and write/ (FETCH_SIZE and WRITE_SIZE
    runs of `bench.py --steps 1 --warmup 0`, copy and TTM kernels only)."""
    import csv
    import glob
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stats = glob.glob(os.path.join(d, "trace", "*kernel_stats.csv"))
    if stats:
        rows = list(csv.DictReader(open(stats[0])))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines = ["kernel time of `bench.py --steps 3 --warmup 1 --no-cpu-baseline` (c2), top kernels",
                 "command: cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run "
                 "-- python3 -u <repo>/bench.py --steps 3 --warmup 1 --no-cpu-baseline",
                 "", f"{'total ms':>10} {'calls':>6} {'avg us':>10}  kernel"]
        for r in rows[:25]:
            lines.append(f"{float(r['TotalDurationNs']) / 1e6:10.3f} {int(r['Calls']):6d} "
                         f"{float(r['AverageNs']) / 1e3:10.1f}  {r['Name'][:110]}")
        with open(os.path.join(out_dir, "hooi_c2_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    fetch = _counter_rows(glob.glob(os.path.join(d, "fetch", "*counter_collection.csv"))[0])
    write = _counter_rows(glob.glob(os.path.join(d, "write", "*counter_collection.csv"))[0])
    # calibration: the bench's 2 GiB device copies (read 2 GiB, write 2 GiB)
    big = [r for r in fetch if r["kernel"] == COPY_KERNEL and r["value"] > 1e6]
    bigw = [r for r in write if r["kernel"] == COPY_KERNEL and r["value"] > 1e6]
    copy_kib = COPY_BYTES / 1024
    f_scale = copy_kib / (sum(r["value"] for r in big) / len(big))
    w_scale = copy_kib / (sum(r["value"] for r in bigw) / len(bigw))
    tf = [r["value"] for r in fetch if TTM_KERNEL in r["kernel"]]
    tw = [r["value"] for r in write if TTM_KERNEL in r["kernel"]]
    per_mode = [round((a * f_scale + b * w_scale) * 1024) for a, b in zip(tf, tw)]
    res = {"kernel": TTM_KERNEL, "workload": "c2 (68,154,792 merged nonzeros, ranks 10), one launch per mode",
           "source_sha256": _sha256(TTM_SOURCE),
           "fetch_kib_per_mode": tf, "write_kib_per_mode": tw,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": sum(r["value"] for r in big) / len(big),
                                "write_kib": sum(r["value"] for r in bigw) / len(bigw),
                                "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
           "hbm_bytes_per_mode": per_mode,
           "commands": ["cd /tmp && rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'k_ttm3_mfma|copyBuffer' "
                        "--output-format csv -d <dir>/fetch -o run -- python3 -u <repo>/bench.py --steps 1 "
                        "--warmup 0 --no-cpu-baseline",
                        "cd /tmp && rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'k_ttm3_mfma|copyBuffer' "
                        "--output-format csv -d <dir>/write -o run -- python3 -u <repo>/bench.py --steps 1 "
                        "--warmup 0 --no-cpu-baseline"]}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))
    # further counter passes of the same command (pmc_*/ directories): the
    # average per TTM launch and per 2 GiB copy of each counter
    lines = []
    for sub in sorted(glob.glob(os.path.join(d, "pmc_*"))):
        files = glob.glob(os.path.join(sub, "*counter_collection.csv"))
        if not files:
            continue
        acc = {}
        for r in csv.DictReader(open(files[0])):
            kern = "ttm" if TTM_KERNEL in r["Kernel_Name"] else ("copy" if r["Kernel_Name"] == COPY_KERNEL else None)
            if kern is None:
                continue
            key = (r["Counter_Name"], kern, int(r["Dispatch_Id"]))
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        names = sorted({k[0] for k in acc})
        cmd = open(os.path.join(sub, "command.txt")).read().strip() if os.path.exists(
            os.path.join(sub, "command.txt")) else ""
        lines.append(f"pass {os.path.basename(sub)}: {cmd}")
        for nm in names:
            for kern in ("ttm", "copy"):
                vals = [v for (c, k, _), v in acc.items() if c == nm and k == kern]
                if kern == "copy":
                    vals = [v for v in vals if v > 0.5 * max(vals, default=0)]   # the 2 GiB copies
                if vals:
                    lines.append(f"  {nm:36s} {kern:5s} mean {sum(vals) / len(vals):16.1f} over {len(vals)} launches")
    if lines:
        hdr = [f"{TTM_KERNEL} counters, c2 (68,154,792 merged nonzeros, ranks 10); 'ttm' = one launch per mode",
               f"(mean over the launches), 'copy' = the bench's 2 GiB device copy.  source sha256 "
               f"{_sha256(TTM_SOURCE)}", ""]
        with open(os.path.join(out_dir, "ttm3_mfma_c2_counters.txt"), "w") as f:
            f.write("\n".join(hdr + lines) + "\n")


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


def cpu_baseline(w, target_s=15.0):
    """The oracle's TTM-chain (FP64, NumPy) on the first nonzeros of the same
    workload, grown until it runs for about target_s seconds."""
    from oracle import ttm
    dims = w["dims"]
    F = w["F0"]
    nnz_total = len(w["vals"])
    n_s = 200_000
    elapsed = 0.0
    while True:
        sl = slice(0, min(n_s, nnz_total))
        idx = [i[sl] for i in w["idx"]]
        vals = w["vals"][sl]
        t0 = time.perf_counter()
        ttm.ttm_chain(idx, vals, F, 0, dims)
        elapsed = time.perf_counter() - t0
        if elapsed >= target_s / 4 or n_s >= nnz_total:
            break
        n_s = int(n_s * min(8.0, max(2.0, target_s / 4 / max(elapsed, 1e-3))))
    return {"value": round(len(vals) / elapsed / 1e9, 6), "unit": "Gnnz/s/mode", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy TTM-chain along mode 1 over the first {len(vals)} drawn nonzeros of the same "
                      f"workload (duplicates not merged), {elapsed:.1f} s on one host thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--share", type=int, default=1, help="one GPU's share of the workload's draws (dims kept)")
    ap.add_argument("--wg-nnz", type=int, default=0, help="elements per Lite bin (0 = library default)")
    ap.add_argument("--rows-cap", type=int, default=0, help="LDS rows per Lite bin (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-profile", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design in DESIGN.md",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import synth
    import paper_1804_09494_amd as P

    torch.cuda.set_device(0)
    t = time.perf_counter()
    w = synth.make_workload(args.workload, scale=args.scale, share=args.share)
    gen_s = time.perf_counter() - t
    dims, ranks = w["dims"], w["ranks"]
    N = len(dims)
    print(f"# generated {args.workload} dims={dims} nnz={len(w['vals'])} in {gen_s:.1f}s", file=sys.stderr,
          flush=True)

    idx_d = [torch.from_numpy(i).cuda() for i in w["idx"]]
    vals_d = torch.from_numpy(w["vals"]).cuda()
    opts = {}
    if args.wg_nnz:
        opts["wg_nnz_target"] = args.wg_nnz
    if args.rows_cap:
        opts["lds_rows_cap"] = args.rows_cap
    ctx = P.TuckerContext(0, **opts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.load_coo(idx_d, vals_d, dims)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t
    del idx_d, vals_d
    t = time.perf_counter()
    ctx.set_ranks(ranks)
    torch.cuda.synchronize()
    part_s = time.perf_counter() - t
    for n, F in enumerate(w["F0"]):
        ctx.set_factor(n, np.ascontiguousarray(F))
    m, _ = ctx.tensor_info()
    print(f"# coalesced m'={m} load {load_s:.2f}s partition+layout {part_s:.2f}s", file=sys.stderr, flush=True)

    copy_gbs = device_copy_bandwidth(torch)
    K = args.steps

    def run(prec):
        """Warm-up invocations, then K timed invocations from the initial factors."""
        ctx.set_options(prec=prec, refine=1)
        for n, F in enumerate(w["F0"]):
            ctx.set_factor(n, np.ascontiguousarray(F))
        if args.warmup > 0:
            ctx.hooi_iterate(args.warmup)
        for n, F in enumerate(w["F0"]):
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
    mfma_path = N == 3 and all(ranks[j] <= 16 for j in range(N))
    # the committed counter summary is of this kernel on c2 as a whole
    traffic = committed_traffic() if (args.workload == "c2" and args.share == 1 and args.scale == 1.0
                                      and mfma_path) else None
    stats = [ctx.partition_stats(n) for n in range(N)]
    print(f"# fits fp32 {fits}", file=sys.stderr, flush=True)
    print(f"# fits bf16 {bf_fits}", file=sys.stderr, flush=True)
    print(f"# per-step ms fp32: " + ", ".join(f"{k}={v / K:.3f}" for k, v in tm.items()), file=sys.stderr, flush=True)
    print(f"# per-step ms bf16: " + ", ".join(f"{k}={v / K:.3f}" for k, v in bf_tm.items()), file=sys.stderr,
          flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)

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
                               f"{N}-mode {'x'.join(str(d) for d in dims)}, "
                               f"{len(w['vals'])} Zipf-drawn nonzeros ({m} after merging), ranks "
                               f"{'x'.join(str(k) for k in ranks)}, one HOOI invocation per step",
                   "m_coalesced": m, "ranks": list(ranks)},
        "hooi_iter_ms": {"fp32": round(ms_per_step, 4), "bf16_gram": round(bf_ms, 4)},
        "bf16_gram_run": f"{K - 1} invocations with BF16 Gram operands, then one refining FP32 invocation",
        "final_fit": {"fp32": fits[-1] if fits else None, "bf16_gram": bf_fits[-1] if bf_fits else None},
        "step_ms_bf16_gram": {k: round(v / K, 4) for k, v in bf_tm.items()},
        "ttm_ms_per_mode": [round(x, 4) for x in ttm_ms],
        "ttm_kernel_ms_per_mode": [round(x, 4) for x in kern_ms],
        "step_ms": {k: round(v / K, 4) for k, v in tm.items()},
        "partition_s": round(part_s, 3),
        "partition_stats": stats,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(float(np.mean(traffic))) if traffic else None,
                     "traffic_bytes_per_mode": traffic,
                     "kernel": "k_ttm3_mfma (TTM-chain)" if mfma_path else "k_ttm (TTM-chain, vector ALU)",
                     "bytes_per_launch": [int(b) for b in B]},
        "device_copy_GBps": round(copy_gbs, 1),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
