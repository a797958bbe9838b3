"""Benchmark of the layered GEMM on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: FP32 SGEMM, M = N = K = 8192, row-major NN, alpha = 1.5, beta = 0.5,
A, B, C entries i.i.d. uniform[-1, 1] (seeded, synthetic).  One step is one
full GEMM C <- alpha*A*B + beta*C on the FP32-MFMA path with all operands
resident in HBM.  The same problem is also timed on the bf16x3 split path
(FP32 accuracy from BF16 matrix cores) for the speedup figure.

Prints one JSON line.  `value` is FP32 TFLOP/s = 2*M*N*K / (mean step time).
`roofline` reports the dominant kernel (the FP32 GEMM kernel) against the FP32
MFMA peak, from per-launch HIP events on the launch stream.  `cpu_baseline`
times the FP64 oracle on a bounded sample of the same GEMM (a block of output
rows) on the host cores, and the same sample gives the sampled normalised error
of each GPU path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "GEMM TFLOP/s & % MFMA peak at 8192³; bf16x3 vs FP32 speedup at ≤1e-5 rel err"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
M = N = K = 8192
ALPHA, BETA = 1.5, 0.5
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "sgemm_f32_8192_nn_traffic.md")
PROFILE_SMALLK = os.path.join(ROOT, "profiles", "sgemm_small_k_traffic.md")
SMALLK_SHAPE = (8192, 8192, 256)
KERNEL_SOURCES = ["paper_2305_18236_amd/csrc/gemm_f32.hip", "paper_2305_18236_amd/csrc/tile_f32.h",
                  "paper_2305_18236_amd/csrc/common.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(profile=PROFILE_TRAFFIC):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(profile):
        return None
    vals = {}
    for line in open(profile):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_path(path, A, B, C, steps, warmup, torch, native):
    """Run `warmup` + `steps` GEMMs on the current stream; per-launch HIP events."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    pid = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}[path]
    need = native.mg_gemm_workspace_size(pid, "N", "N", M, N, K)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)

    def launch():
        st = native.mg_gemm(pid, "N", "N", M, N, K, ALPHA, A.data_ptr(), K, B.data_ptr(), N, BETA,
                            C.data_ptr(), N, ws.data_ptr(), need, sp)
        native.check(st, "mg_gemm")

    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        launch()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    total_ms = ev[0].elapsed_time(ev[steps])
    return {"ms_per_step": total_ms / steps, "kernel_ms_mean": float(np.mean(per)),
            "kernel_ms_median": float(np.median(per)), "kernel_ms_ci95": ci95(per), "wall_s": wall}


def ci95(samples):
    """95 % confidence interval of the mean of per-step times (Student t), the
    statistic the paper reports over its repeated runs; None below 2 samples."""
    n = len(samples)
    if n < 2:
        return None
    m = float(np.mean(samples))
    sd = float(np.std(samples, ddof=1))
    try:
        from scipy.stats import t as student_t
        q = float(student_t.ppf(0.975, n - 1))
    except ImportError:
        q = 1.96
    h = q * sd / np.sqrt(n)
    return [round(float(m - h), 5), round(float(m + h), 5)]


def single_result(path, A, B, C0_dev, torch, native):
    """One GEMM from the original C0 (for the error check)."""
    C = C0_dev.clone()
    pid = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}[path]
    need = native.mg_gemm_workspace_size(pid, "N", "N", M, N, K)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    st = native.mg_gemm(pid, "N", "N", M, N, K, ALPHA, A.data_ptr(), K, B.data_ptr(), N, BETA,
                        C.data_ptr(), N, ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    native.check(st, "mg_gemm")
    torch.cuda.synchronize()
    return C


def cpu_baseline(A_h, B_h, C0_h, gpu_rows, target_s=25.0):
    """Time the FP64 oracle on a block of output rows of the same GEMM, and
    score the GPU results on those rows."""
    import oracle
    threads = oracle.max_threads()
    # calibrate on one row, then size the block to about target_s seconds
    t0 = time.perf_counter()
    oracle.gemm("N", "N", 1, N, K, ALPHA, A_h[:K], K, B_h, N, BETA, C0_h[:N], N, threads=threads)
    t1 = time.perf_counter() - t0
    rows = int(max(threads, min(512, target_s / max(t1, 1e-6) * threads / 2)))
    rows = max(threads, (rows // threads) * threads)
    t0 = time.perf_counter()
    Cref, D = oracle.gemm("N", "N", rows, N, K, ALPHA, A_h[: rows * K], K, B_h, N, BETA,
                          C0_h[: rows * N], N, threads=threads)
    dt = time.perf_counter() - t0
    errs = {p: oracle.normalized_error(g[:rows].astype(np.float64), Cref, D) for p, g in gpu_rows.items()}
    return {"value": 2.0 * rows * N * K / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {rows} of {M} output rows of the same 8192^3 GEMM "
                      f"({rows * N} outputs, full K), FP64 triple loop, {dt:.1f} s"}, errs, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["sgemm", "batched", "chain", "fp8", "sweep", "tiling", "engine", "types", "syr2k",
                             "smallk"],
                    default="sgemm",
                    help="sgemm: the FP32 8192^3 line (default); batched: 512 uneven problems; "
                         "chain: forward + backward of Y = (X W1) W2; fp8: FP8 path at 8192^3; "
                         "sweep: FP32 shapes x layouts; tiling: Tiling vs Tiling+Packing over sizes; "
                         "engine: vector-ALU vs matrix-core micro-kernel; types: FP16 and INT8 at 8192^3; "
                         "syr2k: SYR2K at N = K = 8192")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build targets one GPU; runs on more than one GPU are not supported "
              "(a GEMM shards as independent output tiles; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import seeded_inputs as si
    from paper_2305_18236_amd import _native
    native = _native
    native.lib()
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return

    if args.workload == "batched":
        return bench_batched(args, torch, si, native, dev)
    if args.workload == "chain":
        return bench_chain(args, torch, si, native, dev)
    if args.workload == "fp8":
        return bench_fp8(args, torch, si, native, dev)
    if args.workload == "sweep":
        return bench_sweep(args, torch, si, native, dev)
    if args.workload == "tiling":
        return bench_tiling(args, torch, si, native, dev)
    if args.workload == "engine":
        return bench_engine(args, torch, si, native, dev)
    if args.workload == "types":
        return bench_types(args, torch, si, native, dev)
    if args.workload == "syr2k":
        return bench_syr2k(args, torch, si, native, dev)
    if args.workload == "smallk":
        return bench_smallk(args, torch, si, native, dev)

    A_h = si.uniform((M, K), si.seed_for(2, "A")).reshape(-1)
    B_h = si.uniform((K, N), si.seed_for(2, "B")).reshape(-1)
    C0_h = si.uniform((M, N), si.seed_for(2, "C")).reshape(-1)
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    C0 = torch.from_numpy(C0_h).to(dev)

    flops = 2.0 * M * N * K
    results = {}
    paths = ["fp32"] + [p for p in ("bf16x3",) if _path_supported(native, p)]
    for path in paths:
        C = C0.clone()
        r = time_path(path, A, B, C, args.steps, args.warmup, torch, native)
        r["tflops"] = flops / (r["ms_per_step"] * 1e-3) / 1e12
        r["kernel_tflops"] = flops / (r["kernel_ms_mean"] * 1e-3) / 1e12
        results[path] = r
        del C

    f32 = results["fp32"]
    peak = PEAK_TFLOPS["fp32"]
    achieved = f32["kernel_tflops"]
    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": round(f32["tflops"], 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sgemm_fp32_8192x8192x8192_nn", "M": M, "N": N, "K": K,
                   "layout": "NN", "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]",
                   "path": "fp32"},
        "pct_fp32_mfma_peak": round(100.0 * f32["tflops"] / peak, 2),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                     "kernel": "sgemm_mfma_kernel<256,256,16,128,64,NN>",
                     "kernel_ms_mean": round(f32["kernel_ms_mean"], 4),
                     "algorithmic_flops_per_launch": flops},
    }
    out["step_time_ms"] = {p: {"median": round(r["kernel_ms_median"], 5), "mean": round(r["kernel_ms_mean"], 5),
                               "ci95": r["kernel_ms_ci95"]} for p, r in results.items()}
    if "bf16x3" in results:
        b = results["bf16x3"]
        out["bf16x3"] = {"tflops": round(b["tflops"], 2), "ms_per_step": round(b["ms_per_step"], 4),
                         "speedup_vs_fp32": round(b["tflops"] / f32["tflops"], 3),
                         "pct_bf16_mfma_peak_issued": round(100.0 * 3 * b["tflops"] / PEAK_TFLOPS["bf16"], 2)}

    if not args.no_cpu_baseline:
        rows_needed = 512
        gpu_rows = {}
        for path in results:
            Cp = single_result(path, A, B, C0, torch, native)
            gpu_rows[path] = Cp[: rows_needed * N].cpu().numpy().reshape(rows_needed, N)
        cb, errs, rows = cpu_baseline(A_h, B_h, C0_h, gpu_rows)
        out["cpu_baseline"] = cb
        out["sampled_error_vs_fp64_oracle"] = {p: float(f"{e:.3e}") for p, e in errs.items()}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_batched(args, torch, si, native, dev):
    """512 GEMMs with M, N, K log-uniform in [32, 2048] (multiples of 8), U[-1, 1]:
    one persistent launch against one launch per problem."""
    sizes = si.batched_sizes(512, si.seed_for(4, "A"))
    ops = []
    for i, (m, n, k) in enumerate(sizes):
        A = torch.from_numpy(si.uniform((m, k), si.seed_for(4, "A", i))).to(dev)
        B = torch.from_numpy(si.uniform((k, n), si.seed_for(4, "B", i))).to(dev)
        ops.append((A, B, torch.zeros((m, n), device=dev)))
    flops = sum(2.0 * m * n * k for m, n, k in sizes)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    out = {"metric": "uneven batched GEMM TFLOP/s, 512 problems in one persistent launch",
           "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "batched_uneven_512", "problems": 512,
                      "sizes": "M,N,K log-uniform in [32, 2048], multiples of 8", "layout": "NN",
                      "alpha": 1.0, "beta": 0.0, "total_gflop": round(flops / 1e9, 2)},
           "paths": {}}
    for path in ("fp32", "bf16x3"):
        pid = {"fp32": 0, "bf16x3": 1}[path]
        arr = (native.mg_problem * len(ops))()
        for i, (A, B, C) in enumerate(ops):
            m, k = A.shape
            n = B.shape[1]
            arr[i] = native.mg_problem(b"N", b"N", m, n, k, 1.0, 0.0, A.data_ptr(), k, B.data_ptr(), n,
                                       C.data_ptr(), n)
        need = native.mg_gemm_batched_workspace_size(pid, len(ops))
        ws = torch.empty(need, dtype=torch.uint8, device=dev)

        def persistent():
            st, bad = native.mg_gemm_batched(pid, len(ops), arr, ws.data_ptr(), need, sp)
            native.check(st, "mg_gemm_batched")

        def per_problem():
            for A, B, C in ops:
                m, k = A.shape
                n = B.shape[1]
                native.check(native.mg_gemm(pid, "N", "N", m, n, k, 1.0, A.data_ptr(), k, B.data_ptr(), n,
                                            0.0, C.data_ptr(), n, None, 0, sp), "mg_gemm")

        res = {}
        for name, fn in (("persistent", persistent), ("per_problem", per_problem)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            res[name] = {"ms": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                         "launches": 1 if name == "persistent" else len(ops)}
        res["speedup_persistent_vs_per_problem"] = round(res["per_problem"]["ms"] / res["persistent"]["ms"], 3)
        res["persistent"].update(_batched_tail(native, torch, pid, arr, len(ops), ws, need, sp, dev))
        out["paths"][path] = res
    out["value"] = out["paths"]["fp32"]["persistent"]["tflops"]
    out["ms_per_step"] = out["paths"]["fp32"]["persistent"]["ms"]
    out["dtype"] = "f32"
    print(json.dumps(out), flush=True)


def _batched_tail(native, torch, pid, arr, count, ws, need, sp, dev):
    """One more persistent launch with per-workgroup wall-clock stamps: how
    long the workgroups that found the work list empty waited for the last
    tiles.  tail_idle_frac = sum over workgroups of (last end - own end) over
    workgroups x (last end - first start)."""
    slots = native.mg_batched_slots(pid)
    stamps = torch.zeros(2 * slots, dtype=torch.int64, device=dev)
    st, bad, grid = native.mg_gemm_batched_timed(pid, count, arr, ws.data_ptr(), need, sp, stamps.data_ptr(),
                                                 2 * slots)
    native.check(st, "mg_gemm_batched_timed")
    torch.cuda.synchronize()
    t = stamps.cpu().view(-1, 2)[:grid].double()
    hz = float(native.mg_wall_clock_hz())
    t0, t1 = float(t[:, 0].min()), float(t[:, 1].max())
    ends = t[:, 1]
    return {"workgroups": grid,
            "stamped_span_us": round((t1 - t0) / hz * 1e6, 1),
            "tail_us": round((t1 - float(ends.min())) / hz * 1e6, 1),
            "median_end_to_last_us": round((t1 - float(ends.median())) / hz * 1e6, 1),
            "tail_idle_frac": round(float((t1 - ends).sum()) / (grid * (t1 - t0)), 4)}


def bench_chain(args, torch, si, native, dev):
    """Y = (X W1) W2 with X 4096x2048, W1 2048x8192, W2 8192x2048; one step is
    the forward (2 GEMMs) and the hand-written backward (4 GEMMs) of
    loss = sum(Y * G), on the bf16x3 path and on the FP32 path."""
    from paper_2305_18236_amd.autograd import chain
    Mx, D, Hd = 4096, 2048, 8192
    X = torch.from_numpy(si.uniform((Mx, D), si.seed_for(5, "X"))).to(dev).requires_grad_(True)
    W1 = torch.from_numpy(si.uniform((D, Hd), si.seed_for(5, "W1"))).to(dev).requires_grad_(True)
    W2 = torch.from_numpy(si.uniform((Hd, D), si.seed_for(5, "W2"))).to(dev).requires_grad_(True)
    G = torch.from_numpy(si.gaussian((Mx, D), si.seed_for(5, "G"))).to(dev)
    gemm_flop = 2.0 * Mx * D * Hd
    flops = 6 * gemm_flop
    out = {"metric": "differentiable GEMM chain TFLOP/s (forward + hand-written backward)",
           "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "gemm_chain_4096x2048x8192", "X": [Mx, D], "W1": [D, Hd], "W2": [Hd, D],
                      "loss": "sum(Y*G), G ~ N(0,1)", "gemms_per_step": 6,
                      "gflop_per_step": round(flops / 1e9, 1)},
           "paths": {}}
    stream = torch.cuda.current_stream()
    for path in ("bf16x3", "fp32"):
        def step():
            for t in (X, W1, W2):
                t.grad = None
            Y = chain(X, W1, W2, path)
            Y.backward(G)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out["paths"][path] = {"ms_per_step": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2)}
    b, f = out["paths"]["bf16x3"], out["paths"]["fp32"]
    out["value"] = b["tflops"]
    out["ms_per_step"] = b["ms_per_step"]
    out["dtype"] = "bf16x3"
    out["speedup_bf16x3_vs_fp32"] = round(f["ms_per_step"] / b["ms_per_step"], 3)
    print(json.dumps(out), flush=True)


def _time_ms(fn, steps, warmup, torch, stream, min_warm_ms=150.0):
    """Mean time of `steps` back-to-back calls on `stream` (HIP events).

    Warm-up runs `warmup` calls and then keeps going until the warm-up has
    taken `min_warm_ms` of wall time: after the host has prepared fresh inputs
    the GPU has idled and its clock ramps back up over tens of milliseconds,
    which would otherwise be charged to the first timed case."""
    t0 = time.perf_counter()
    n = 0
    while n < warmup or (time.perf_counter() - t0) * 1e3 < min_warm_ms:
        fn()
        n += 1
        if n >= warmup:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _time_per_launch_ms(fn, steps, warmup, torch, stream, min_warm_ms=150.0):
    """Median over `steps` calls of the time between HIP events recorded just
    before and just after each call on `stream`.  For launches of a few
    microseconds a back-to-back loop measures the launch rate of the host;
    the events bracket the call's own work on the GPU."""
    _time_ms(fn, 1, warmup, torch, stream, min_warm_ms)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return t[len(t) // 2]


def bench_fp8(args, torch, si, native, dev):
    """The FP8 path at 8192^3 (NN, alpha 1, beta 0, U[-1, 1]): the two pack
    (quantise) launches, the GEMM on packed operands alone, and the whole
    mg_gemm call; plus the plain BF16 path for reference."""
    A = torch.from_numpy(si.uniform((M, K), si.seed_for(3, "A"))).to(dev)
    B = torch.from_numpy(si.uniform((K, N), si.seed_for(3, "B"))).to(dev)
    C = torch.zeros((M, N), device=dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    qa_b, sa_b = native.mg_fp8_packed_size(M, K)
    qb_b, sb_b = native.mg_fp8_packed_size(N, K)
    qA = torch.empty(qa_b, dtype=torch.uint8, device=dev)
    sA = torch.empty(sa_b, dtype=torch.uint8, device=dev)
    qB = torch.empty(qb_b, dtype=torch.uint8, device=dev)
    sB = torch.empty(sb_b, dtype=torch.uint8, device=dev)
    need = native.mg_gemm_workspace_size(3, "N", "N", M, N, K)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def pack():
        native.check(native.mg_fp8_pack("N", M, K, A.data_ptr(), K, qA.data_ptr(), sA.data_ptr(), sp), "pack A")
        native.check(native.mg_fp8_pack("T", N, K, B.data_ptr(), N, qB.data_ptr(), sB.data_ptr(), sp), "pack B")

    def gemm_only():
        native.check(native.mg_gemm_fp8_packed(M, N, K, 1.0, qA.data_ptr(), sA.data_ptr(), qB.data_ptr(),
                                               sB.data_ptr(), 0.0, C.data_ptr(), N, sp), "fp8 gemm")

    def whole(path):
        w = ws if path == 3 else torch.empty(max(native.mg_gemm_workspace_size(path, "N", "N", M, N, K), 1),
                                             dtype=torch.uint8, device=dev)
        n = native.mg_gemm_workspace_size(path, "N", "N", M, N, K)
        return lambda: native.check(native.mg_gemm(path, "N", "N", M, N, K, 1.0, A.data_ptr(), K, B.data_ptr(), N,
                                                   0.0, C.data_ptr(), N, w.data_ptr(), n, sp), "mg_gemm")

    pack()
    flops = 2.0 * M * N * K
    t_pack = _time_ms(pack, args.steps, args.warmup, torch, stream)
    t_gemm = _time_ms(gemm_only, args.steps, args.warmup, torch, stream)
    t_whole = _time_ms(whole(3), args.steps, args.warmup, torch, stream)
    t_bf16 = _time_ms(whole(2), args.steps, args.warmup, torch, stream)
    pack_bytes = 2 * (4.0 + 1.0) * M * K        # read FP32, write E4M3, both operands
    out = {"metric": "FP8 (E4M3, per-128x128-tile scales) GEMM TFLOP/s at 8192^3", "unit": "TFLOP/s",
           "value": round(flops / (t_whole * 1e-3) / 1e12, 2), "ms_per_step": round(t_whole, 4),
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp8_e4m3", "data": "synthetic",
           "config": {"workload": "gemm_fp8_t128_8192x8192x8192_nn", "M": M, "N": N, "K": K, "layout": "NN"},
           "pack_ms": round(t_pack, 4), "pack_gbps": round(pack_bytes / (t_pack * 1e-3) / 1e9, 1),
           "gemm_only_ms": round(t_gemm, 4),
           "gemm_only_tflops": round(flops / (t_gemm * 1e-3) / 1e12, 2),
           "gemm_only_pct_fp8_peak": round(100 * flops / (t_gemm * 1e-3) / 1e12 / PEAK_TFLOPS["fp8"], 2),
           "bf16_tflops": round(flops / (t_bf16 * 1e-3) / 1e12, 2)}
    print(json.dumps(out), flush=True)


SWEEP_SHAPES = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
                (8192, 8192, 256), (256, 8192, 8192), (16384, 1024, 4096),
                # shapes whose workgroups do not fall into whole rounds over the
                # compute units (the FP32 round plan and the 16-bit split rule)
                (1536, 1536, 1536), (3072, 3072, 3072), (6144, 6144, 6144), (3072, 3072, 1024)]


def bench_sweep(args, torch, si, native, dev):
    """The FP32 sweep (alpha 1.5, beta 0.5, U[-1, 1]) in all four layouts on the
    FP32 path, then NN on the bf16x3 path; one JSON line with a row per case.
    The bf16x3 cases run after every FP32 case: the chip clocks down under
    sustained BF16 matrix work and takes a while to recover, which would
    otherwise be charged to the FP32 case that follows."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    rows = []
    for path, layouts in (("fp32", [tA + tB for tA in "NT" for tB in "NT"]), ("bf16x3", ["NN"])):
        pid = {"fp32": 0, "bf16x3": 1}[path]
        for (m, n, k) in SWEEP_SHAPES:
            A = torch.from_numpy(si.uniform((m * k,), si.seed_for(2, "A"))).to(dev)
            B = torch.from_numpy(si.uniform((k * n,), si.seed_for(2, "B"))).to(dev)
            C = torch.from_numpy(si.uniform((m * n,), si.seed_for(2, "C"))).to(dev)
            flops = 2.0 * m * n * k
            for tA, tB in layouts:
                lda = k if tA == "N" else m
                ldb = n if tB == "N" else k
                need = native.mg_gemm_workspace_size(pid, tA, tB, m, n, k)
                ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

                def run():
                    native.check(native.mg_gemm(pid, tA, tB, m, n, k, ALPHA, A.data_ptr(), lda, B.data_ptr(), ldb,
                                                BETA, C.data_ptr(), n, ws.data_ptr(), need, sp), "mg_gemm")

                ms = _time_ms(run, args.steps, args.warmup, torch, stream)
                tf = flops / (ms * 1e-3) / 1e12
                rows.append({"M": m, "N": n, "K": k, "path": path, "layout": tA + tB, "ms": round(ms, 4),
                             "tflops": round(tf, 2),
                             "pct_fp32_peak": round(100 * tf / PEAK_TFLOPS["fp32"], 1) if path == "fp32" else None,
                             "config": native.mg_tuned_config(pid, m, n, k),
                             "splits": native.mg_split_count(pid, m, n, k)})
            del A, B, C
    nn8 = [r for r in rows if r["M"] == 8192 and r["K"] == 8192 and r["path"] == "fp32" and r["layout"] == "NN"][0]
    out = {"metric": "FP32 SGEMM sweep TFLOP/s (all layouts) and bf16x3 NN", "unit": "TFLOP/s",
           "value": nn8["tflops"], "ms_per_step": nn8["ms"], "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sgemm_sweep", "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]"},
           "rows": rows}
    print(json.dumps(out), flush=True)


TILING_SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]


def bench_tiling(args, torch, si, native, dev):
    """The packing ablation of the paper's Section 4.1.3 on the FP32 path:
    square SGEMMs C = A B (NN, alpha 1, beta 0) over the paper's sizes, each
    timed with every tile configuration; "Tiling" is the best configuration
    that loads operands straight into registers, "Tiling+Packing" the best one
    that packs them into LDS (split-K allowed for both, as the library would
    run them).  One JSON line with a row per size."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    ncfg = native.mg_num_configs(0)
    rows = []
    for n in TILING_SIZES:
        A = torch.from_numpy(si.uniform((n * n,), si.seed_for(2, "A"))).to(dev)
        B = torch.from_numpy(si.uniform((n * n,), si.seed_for(2, "B"))).to(dev)
        C = torch.zeros(n * n, device=dev)
        steps = max(args.steps, 200 if n <= 512 else 20)
        per_cfg = {}
        for cfg in range(ncfg):
            native.check(native.mg_force_config(0, cfg), "mg_force_config")
            try:
                need = native.mg_gemm_workspace_size(0, "N", "N", n, n, n)
                ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

                def run():
                    native.check(native.mg_gemm(0, "N", "N", n, n, n, 1.0, A.data_ptr(), n, B.data_ptr(), n, 0.0,
                                                C.data_ptr(), n, ws.data_ptr(), need, sp), "mg_gemm")

                per_cfg[cfg] = _time_per_launch_ms(run, steps, args.warmup, torch, stream)
            finally:
                native.mg_force_config(0, -1)
        flops = 2.0 * n ** 3
        best = {}
        for name, packs in (("tiling", 0), ("tiling_packing", 1)):
            cands = {c: t for c, t in per_cfg.items() if native.mg_config_packs(0, c) == packs}
            c = min(cands, key=cands.get)
            best[name] = {"config": c, "us": round(cands[c] * 1e3, 2),
                          "tflops": round(flops / (cands[c] * 1e-3) / 1e12, 3)}
        rows.append({"M": n, "N": n, "K": n, **best,
                     "packing_speedup": round(best["tiling"]["us"] / best["tiling_packing"]["us"], 3),
                     "auto_config": native.mg_tuned_config(0, n, n, n)})
        del A, B, C
    big = rows[-1]
    out = {"metric": "FP32 SGEMM time, Tiling vs Tiling+Packing over sizes", "unit": "TFLOP/s",
           "value": big["tiling_packing"]["tflops"], "ms_per_step": big["tiling_packing"]["us"] / 1e3,
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sgemm_packing_ablation", "alpha": 1.0, "beta": 0.0, "layout": "NN",
                      "inputs": "uniform[-1,1]", "timing": "median over launches of HIP events recorded around each call"},
           "rows": rows}
    print(json.dumps(out), flush=True)


ENGINE_SIZES = [1024, 2048, 4096, 8192]
# FP32 on the vector ALUs: the published 157.3 TFLOP/s (256 flop per clock per
# CU at 2.4 GHz).  The kernels issue scalar v_fmac_f32 only (packed FP32 is
# disabled at build time); they measure above 78.6 TFLOP/s, so scalar FMAs are
# not limited to half the vector rate on this chip and the full figure is the
# bound.
VALU_FP32_PEAK = 256 * 256 * 2.4e9 / 1e12


def bench_engine(args, torch, si, native, dev):
    """The paper's generic-vs-MMA lowering comparison (Section 4.4) on the GPU:
    the same packed macro level with the vector-ALU FMA micro-kernel and with
    the MFMA micro-kernel, square FP32 SGEMMs (NN, alpha 1.5, beta 0.5).  MFMA
    runs the automatic configuration; VALU the best of its configurations."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    ncfg = native.mg_num_configs(0)
    valu_cfgs = [c for c in range(ncfg) if native.mg_config_uses_mfma(0, c) == 0]
    rows = []
    for n in ENGINE_SIZES:
        A = torch.from_numpy(si.uniform((n * n,), si.seed_for(2, "A"))).to(dev)
        B = torch.from_numpy(si.uniform((n * n,), si.seed_for(2, "B"))).to(dev)
        C = torch.from_numpy(si.uniform((n * n,), si.seed_for(2, "C"))).to(dev)
        steps = args.steps if n >= 4096 else max(args.steps, 50)

        def timed(cfg):
            if cfg is not None:
                native.check(native.mg_force_config(0, cfg), "mg_force_config")
            try:
                need = native.mg_gemm_workspace_size(0, "N", "N", n, n, n)
                ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

                def run():
                    native.check(native.mg_gemm(0, "N", "N", n, n, n, ALPHA, A.data_ptr(), n, B.data_ptr(), n, BETA,
                                                C.data_ptr(), n, ws.data_ptr(), need, sp), "mg_gemm")

                return _time_ms(run, steps, args.warmup, torch, stream)
            finally:
                native.mg_force_config(0, -1)

        valu = {c: timed(c) for c in valu_cfgs}
        vc = min(valu, key=valu.get)
        mfma_ms = timed(None)
        flops = 2.0 * n ** 3
        tf_v, tf_m = flops / (valu[vc] * 1e-3) / 1e12, flops / (mfma_ms * 1e-3) / 1e12
        rows.append({"M": n, "N": n, "K": n,
                     "valu": {"config": vc, "ms": round(valu[vc], 4), "tflops": round(tf_v, 2),
                              "frac_of_valu_peak": round(tf_v / VALU_FP32_PEAK, 3)},
                     "mfma": {"config": native.mg_tuned_config(0, n, n, n), "ms": round(mfma_ms, 4),
                              "tflops": round(tf_m, 2), "frac_of_mfma_peak": round(tf_m / PEAK_TFLOPS["fp32"], 3)},
                     "mfma_speedup": round(valu[vc] / mfma_ms, 3)})
        del A, B, C
    big = rows[-1]
    out = {"metric": "FP32 SGEMM TFLOP/s, vector-ALU vs matrix-core micro-kernel", "unit": "TFLOP/s",
           "value": big["valu"]["tflops"], "ms_per_step": big["valu"]["ms"], "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sgemm_valu_vs_mfma", "alpha": ALPHA, "beta": BETA, "layout": "NN",
                      "inputs": "uniform[-1,1]"},
           "roofline": {"bound": "alu", "achieved": big["valu"]["tflops"], "peak": round(VALU_FP32_PEAK, 1),
                        "unit": "TFLOP/s", "frac": big["valu"]["frac_of_valu_peak"], "traffic": None,
                        "kernel": f"sgemm_valu_kernel (config {big['valu']['config']}) at 8192^3"},
           "rows": rows}
    print(json.dumps(out), flush=True)


INT8_PEAK_TOPS = 5033.2


def bench_types(args, torch, si, native, dev):
    """Table 1's other operand types at 8192^3 NN: the FP16 path (FP32
    operands rounded to binary16, end to end) and the INT8 entry points (int8
    operands, int32 C; end to end including the pack, and the GEMM alone on
    packed operands).  alpha 1, beta 0 (INT8: alpha 1, beta 0)."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    n = M
    flops = 2.0 * n ** 3
    A = torch.from_numpy(si.uniform((n * n,), si.seed_for(3, "A"))).to(dev)
    B = torch.from_numpy(si.uniform((n * n,), si.seed_for(3, "B"))).to(dev)
    C = torch.zeros(n * n, device=dev)
    need = native.mg_gemm_workspace_size(4, "N", "N", n, n, n)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

    def fp16():
        native.check(native.mg_gemm(4, "N", "N", n, n, n, 1.0, A.data_ptr(), n, B.data_ptr(), n, 0.0,
                                    C.data_ptr(), n, ws.data_ptr(), need, sp), "mg_gemm")

    fp16_ms = _time_ms(fp16, args.steps, args.warmup, torch, stream)
    del A, B, C, ws
    g = torch.Generator(device=dev)
    g.manual_seed(si.seed_for(3, "A"))
    Ai = torch.randint(-128, 128, (n * n,), dtype=torch.int8, device=dev, generator=g)
    Bi = torch.randint(-128, 128, (n * n,), dtype=torch.int8, device=dev, generator=g)
    Ci = torch.zeros(n * n, dtype=torch.int32, device=dev)
    need = native.mg_gemm_i8_workspace_size(n, n, n)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def i8_full():
        native.check(native.mg_gemm_i8("N", "N", n, n, n, 1, Ai.data_ptr(), n, Bi.data_ptr(), n, 0, Ci.data_ptr(),
                                       n, ws.data_ptr(), need, sp), "mg_gemm_i8")

    i8_ms = _time_ms(i8_full, args.steps, args.warmup, torch, stream)
    q = native.mg_i8_packed_size(n, n)
    qA, qB = ws[:q], ws[need - q:]

    def i8_gemm():
        native.check(native.mg_gemm_i8_packed(n, n, n, 1, qA.data_ptr(), qB.data_ptr(), 0, Ci.data_ptr(), n, sp),
                     "mg_gemm_i8_packed")

    i8g_ms = _time_ms(i8_gemm, args.steps, args.warmup, torch, stream)
    rows = {
        "fp16": {"ms": round(fp16_ms, 4), "tflops": round(flops / fp16_ms / 1e9, 1),
                 "frac_of_fp16_peak": round(flops / fp16_ms / 1e9 / PEAK_TFLOPS["bf16"], 3),
                 "config": native.mg_tuned_config(4, n, n, n)},
        "int8_end_to_end": {"ms": round(i8_ms, 4), "tops": round(flops / i8_ms / 1e9, 1),
                            "frac_of_int8_peak": round(flops / i8_ms / 1e9 / INT8_PEAK_TOPS, 3)},
        "int8_gemm_only": {"ms": round(i8g_ms, 4), "tops": round(flops / i8g_ms / 1e9, 1),
                           "frac_of_int8_peak": round(flops / i8g_ms / 1e9 / INT8_PEAK_TOPS, 3),
                           "config": native.mg_tuned_config(5, n, n, n)},
    }
    out = {"metric": "FP16 TFLOP/s and INT8 TOP/s at 8192^3", "unit": "TOP/s",
           "value": rows["int8_gemm_only"]["tops"], "ms_per_step": rows["int8_gemm_only"]["ms"], "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "i8", "data": "synthetic",
           "config": {"workload": "fp16_int8_8192x8192x8192_nn", "fp16_inputs": "uniform[-1,1] float32",
                      "int8_inputs": "uniform integers in [-128, 127]"},
           "roofline": {"bound": "mfma", "achieved": rows["int8_gemm_only"]["tops"], "peak": INT8_PEAK_TOPS,
                        "unit": "TOP/s", "frac": rows["int8_gemm_only"]["frac_of_int8_peak"], "traffic": None,
                        "kernel": "gemm_i8_direct_kernel<256,256,128,64>"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def bench_smallk(args, torch, si, native, dev):
    """The small-K shape of the FP32 sweep, 8192 x 8192 x 256 NN (alpha 1.5,
    beta 0.5, U[-1, 1]), on the FP32 and bf16x3 paths.  Algorithmic HBM bytes
    per launch: 4(MK + KN) + 8MN (A and B read once, C0 read, C written);
    at 62 flop per byte the shape is still matrix-core bound on paper (ridge
    19.7 flop/B for FP32), but its K loop is 8 panels deep (BK = 32), so the
    epilogue's C traffic weighs 32 times more than at K = 8192."""
    m, n, k = SMALLK_SHAPE
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    A = torch.from_numpy(si.uniform((m * k,), si.seed_for(2, "A"))).to(dev)
    B = torch.from_numpy(si.uniform((k * n,), si.seed_for(2, "B"))).to(dev)
    C0 = torch.from_numpy(si.uniform((m * n,), si.seed_for(2, "C"))).to(dev)
    flops = 2.0 * m * n * k
    nbytes = 4.0 * (m * k + k * n) + 8.0 * m * n
    rows = {}
    for name, pid in (("fp32", 0), ("bf16x3", 1)):
        C = C0.clone()
        need = native.mg_gemm_workspace_size(pid, "N", "N", m, n, k)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

        def run():
            native.check(native.mg_gemm(pid, "N", "N", m, n, k, ALPHA, A.data_ptr(), k, B.data_ptr(), n, BETA,
                                        C.data_ptr(), n, ws.data_ptr(), need, sp), "mg_gemm")

        ms = _time_ms(run, args.steps, args.warmup, torch, stream)
        rows[name] = {"ms": round(ms, 4), "tflops": round(flops / ms / 1e9, 2),
                      "algorithmic_gbps": round(nbytes / ms / 1e6, 1), "config": native.mg_tuned_config(pid, m, n, k)}
        del C, ws
    f = rows["fp32"]
    traffic = measured_traffic(PROFILE_SMALLK)
    out = {"metric": "FP32 SGEMM TFLOP/s and HBM GB/s at 8192x8192x256", "unit": "TFLOP/s", "value": f["tflops"],
           "ms_per_step": f["ms"], "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sgemm_small_k_8192x8192x256_nn", "M": m, "N": n, "K": k, "layout": "NN",
                      "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]"},
           "roofline": {"bound": "mfma", "achieved": f["tflops"], "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                        "frac": round(f["tflops"] / PEAK_TFLOPS["fp32"], 4), "traffic": traffic,
                        "kernel": "sgemm_mfma_kernel<128,64,32,64,32,NN>",
                        "algorithmic_bytes_per_launch": nbytes,
                        "hbm_gbps_measured": None if traffic is None else round(traffic / f["ms"] / 1e6, 1)},
           "rows": rows}
    print(json.dumps(out), flush=True)


def bench_syr2k(args, torch, si, native, dev):
    """SYR2K (Section 5.1) on the lower triangle, N = K = 8192, trans 'N',
    alpha 1.5, beta 0.5: one launch over the triangle's tiles, both products
    in one accumulator.  Work counted as 2*N^2*K (the triangle's N(N+1)/2
    entries, two K-long dot products each).  Beside it, the same update done
    with two full FP32 GEMMs (C += alpha*A*B^T, then C += alpha*B*A^T over the
    whole square), the way it would be written without SYR2K."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    n = k = M
    X = torch.from_numpy(si.uniform((n * k,), si.seed_for(5, "X"))).to(dev)
    Y = torch.from_numpy(si.uniform((n * k,), si.seed_for(5, "W1"))).to(dev)
    C = torch.from_numpy(si.uniform((n * n,), si.seed_for(5, "C"))).to(dev)

    need = native.mg_syr2k_workspace_size(0, n, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

    def run(splits):
        native.check(native.mg_force_splits(0, splits), "mg_force_splits")
        try:
            w = native.mg_syr2k_workspace_size(0, n, k)

            def syr2k():
                native.check(native.mg_syr2k(0, "L", "N", n, k, ALPHA, X.data_ptr(), k, Y.data_ptr(), k, BETA,
                                             C.data_ptr(), n, ws.data_ptr(), w, sp), "mg_syr2k")

            return _time_ms(syr2k, args.steps, args.warmup, torch, stream)
        finally:
            native.mg_force_splits(0, -1)

    ms = run(-1)                       # the automatic plan
    auto_splits = need // (4 * n * n) if need else 1
    ms_unsplit = run(1)

    def two_gemms():
        native.check(native.mg_gemm(0, "N", "T", n, n, k, ALPHA, X.data_ptr(), k, Y.data_ptr(), k, BETA,
                                    C.data_ptr(), n, None, 0, sp), "mg_gemm")
        native.check(native.mg_gemm(0, "N", "T", n, n, k, ALPHA, Y.data_ptr(), k, X.data_ptr(), k, 1.0,
                                    C.data_ptr(), n, None, 0, sp), "mg_gemm")

    ms2 = _time_ms(two_gemms, max(2, args.steps // 2), 1, torch, stream)
    flops = 2.0 * n * n * k
    tf = flops / (ms * 1e-3) / 1e12
    out = {"metric": "SYR2K TFLOP/s (2*N^2*K useful flops) at N = K = 8192", "unit": "TFLOP/s",
           "value": round(tf, 2), "ms_per_step": round(ms, 4), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "ssyr2k_lower_n_8192x8192", "N": n, "K": k, "uplo": "L", "trans": "N",
                      "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]"},
           "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                        "frac": round(tf / PEAK_TFLOPS["fp32"], 4), "traffic": None,
                        "kernel": f"syr2k_kernel (config {native.mg_tuned_config(0, n, n, k)} tiles)"},
           "splits": int(auto_splits), "unsplit_ms": round(ms_unsplit, 4),
           "two_full_gemms": {"ms": round(ms2, 4), "speedup_of_syr2k": round(ms2 / ms, 3)}}
    print(json.dumps(out), flush=True)


def _path_supported(native, path) -> bool:
    pid = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}[path]
    return native.mg_num_configs(pid) > 0


if __name__ == "__main__":
    main()
