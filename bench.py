"""Benchmark of the layered GEMM on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload NAME] [--rounds R] [--order-seed S]

Default workload: FP32 SGEMM, M = N = K = 8192, row-major NN, alpha = 1.5,
beta = 0.5, A, B, C entries i.i.d. uniform[-1, 1] (seeded, synthetic).  One
step is one full GEMM C <- alpha*A*B + beta*C on the FP32-MFMA path with all
operands resident in HBM.  The same problem is also timed on the bf16x3 split
path (FP32 accuracy from BF16 matrix cores) for the speedup figure.

Every workload prints one JSON line.  Each timed case carries:
  * its error against the FP64 oracle (max |C - C_ref| / (|alpha||A||B| +
    |beta||C0|) over sampled outputs, corners included; INT8: the number of
    sampled outputs that differ from the exact integer oracle);
  * the shader clock (the spec peaks assume 2.4 GHz; under sustained matrix
    work the chip runs slower), from a probe of 16 one-wave workgroups that
    times the shader-cycle counter against the constant-rate wall clock:
    "during" runs on a second stream while the timed steps are still
    executing (null when the GPU gave it no room before they ended) and
    "after" runs queued right behind them (the clock recovers within
    microseconds of the load ending, so "after" reads high); lists of
    clocks hold one [during, after] pair per timed block;
  * the median and the 95 % confidence interval of its per-step times.
The cases of a workload run in an order shuffled per round (the paper's
randomised run order, Section 4.1.4) by a seeded generator whose seed is
reported.

The oracle runs only in this file's oracle leg (the functions under "oracle
leg" below), on the host, after the GPU timing is done; nothing the GPU times
depends on it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import random
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "GEMM TFLOP/s & % MFMA peak at 8192³; bf16x3 vs FP32 speedup at ≤1e-5 rel err"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
# spec peak of the matrix instructions each path issues, and how many of them
# one useful multiply-add costs (bf16x3: three BF16 products)
DTYPE_PEAK = {"fp32": 157.3, "bf16x3": 2516.6, "bf16": 2516.6, "fp16": 2516.6, "fp8": 5033.2}
ISSUED = {"fp32": 1, "bf16x3": 3, "bf16": 1, "fp16": 1, "fp8": 1}
PATH_ID = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}
TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-2, "fp8": 6e-2, "fp16": 2e-3}
M = N = K = 8192
ALPHA, BETA = 1.5, 0.5
SAMPLES = 1024
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


def tuned_kernel_name(native, path, kernel, M, N, K):
    """`kernel<BM,BN,WM,WN> (configuration c)` for the configuration the
    library picks for an M x N x K GEMM on `path` (the direct-copy kernels'
    template arguments)."""
    cfg = native.mg_tuned_config(path, M, N, K)
    c = native.mg_config_info(path, cfg)
    return f"{kernel}<{c['bm']},{c['bn']},{c['wm']},{c['wn']}> (configuration {cfg})"


def native_plan_config(bench, M, N, K):
    """The FP32 configuration mg_gemm runs for an M x N x K problem (no workspace)."""
    st, cfg, _, _ = bench.native.mg_gemm_plan(PATH_ID["fp32"], M, N, K, 0)
    return cfg if st == 0 else -1


# ------------------------------------------------------------ statistics ---

def ci95(samples):
    """95 % confidence interval of the mean (Student t), the statistic the
    paper reports over its repeated runs; None below 2 samples."""
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


def stats(samples_ms):
    return {"median": round(float(np.median(samples_ms)), 5), "mean": round(float(np.mean(samples_ms)), 5),
            "ci95": ci95(samples_ms), "n": len(samples_ms)}


def tflops(flops, ms):
    return flops / (ms * 1e-3) / 1e12


def progress(msg):
    """One line on stderr as a phase of the run ends (the JSON line is the only stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- timing ---

class Bench:
    """Shared state of a run: the library, the stream, the order generator."""

    def __init__(self, args, torch, native, dev):
        self.args, self.torch, self.native, self.dev = args, torch, native, dev
        self.stream = torch.cuda.current_stream()
        self.sp = self.stream.cuda_stream
        # a second stream (default priority, like the first) for the clock
        # probe that runs beside the timed steps
        self.side = torch.cuda.Stream(device=dev)
        seed = args.order_seed if args.order_seed is not None else int.from_bytes(os.urandom(4), "little")
        self.order_seed = seed
        self.rng = random.Random(seed)

    def shuffled(self, cases):
        cases = list(cases)
        self.rng.shuffle(cases)
        return cases

    def sclk(self):
        """Shader clock (MHz) from a probe queued behind the work on the stream."""
        st, mhz = self.native.mg_shader_clock_mhz(self.sp, 50)
        return round(mhz, 1) if st == 0 else None

    def warm(self, fn, warmup, min_warm_ms=150.0):
        """`warmup` calls, continued until `min_warm_ms` of wall time has passed:
        after the host has prepared inputs the GPU has idled and its clock ramps
        back up over tens of milliseconds, which would otherwise be charged to
        the first timed steps."""
        t0 = time.perf_counter()
        n = 0
        while n < warmup or (time.perf_counter() - t0) * 1e3 < min_warm_ms:
            fn()
            n += 1
            if n >= warmup:
                self.torch.cuda.synchronize()
        self.torch.cuda.synchronize()

    def steps(self, fn, steps, probe=False, calls=1):
        """`steps` samples of `calls` back-to-back calls each, with a HIP
        event between consecutive samples on the launch stream; returns
        (per-call ms of each sample, total ms, clock during the samples).
        probe: once the samples are queued, the clock probe runs on the side
        stream, beside them when the GPU has room for its 16 one-wave
        workgroups; its reading counts as taken during the samples only if
        the launch stream is still busy when it returns."""
        torch = self.torch
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(self.stream)
        for i in range(steps):
            for _ in range(calls):
                fn()
            ev[i + 1].record(self.stream)
        during = None
        if probe:
            st, mhz = self.native.mg_shader_clock_mhz(self.side.cuda_stream, 100)
            if st == 0 and not self.stream.query():
                during = round(mhz, 1)
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) / calls for i in range(steps)]
        return per, ev[0].elapsed_time(ev[steps]), during

    def per_launch(self, fn, steps, between=None):
        """Per-call times from an event pair around each call (for launches of
        a few microseconds, where a back-to-back loop measures the host's
        launch rate); `between` runs before each call, outside the pair."""
        torch = self.torch
        out = []
        for _ in range(steps):
            if between is not None:
                between()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            fn()
            e1.record(self.stream)
            if between is not None:
                torch.cuda.synchronize()
            out.append((e0, e1))
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in out]

    def load_clock(self, fn, per_ms):
        """The clock while fn's kernels run: untimed calls (about 3 ms of
        them) queued after the timed steps, probed from the side stream (see
        steps); None if they finished before the probe returned."""
        n = max(3, min(400, int(3.0 / max(float(np.median(per_ms)), 1e-3))))
        _, _, during = self.steps(fn, n, probe=True)
        return during

    def calls_per_sample(self, fn):
        """Calls per timed sample: 1 for calls of 0.1 ms and more; shorter
        calls are timed in back-to-back blocks of about 0.5 ms, since an
        event between every two calls adds its own gap (a 25 us GEMM: about
        2.5 us) to each."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(4):
            fn()
        e1.record(self.stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 4
        return 1 if t >= 0.1 else max(1, min(200, int(0.5 / max(t, 1e-4))))

    def case(self, fn, steps=None, warmup=None):
        """Warm up, time `steps` samples (single calls, or blocks of calls
        for short ones), read the clock right after them, then the clock
        under the same load (outside the timed samples, so that the probe's
        workgroups never share the GPU with a timed one)."""
        steps = self.args.steps if steps is None else steps
        warmup = self.args.warmup if warmup is None else warmup
        self.warm(fn, warmup)
        calls = self.calls_per_sample(fn)
        per, total, _ = self.steps(fn, steps, calls=calls)
        after = self.sclk()
        return {"per_ms": per, "total_ms": total, "sclk_mhz": after, "calls_per_sample": calls,
                "sclk_mhz_during": self.load_clock(fn, per)}

    def gemm_call(self, path, tA, tB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws=None):
        """A closure launching mg_gemm with its full workspace (allocated here once)."""
        pid = PATH_ID[path]
        need = self.native.mg_gemm_workspace_size(pid, tA, tB, m, n, k)
        if ws is None or ws.numel() < need:
            ws = self.torch.empty(max(need, 1), dtype=self.torch.uint8, device=self.dev)
        native, sp = self.native, self.sp
        a, b, c, w = A.data_ptr(), B.data_ptr(), C.data_ptr(), ws.data_ptr()

        def run():
            native.check(native.mg_gemm(pid, tA, tB, m, n, k, alpha, a, lda, b, ldb, beta, c, ldc, w, need, sp),
                         "mg_gemm")
        run.workspace = ws
        return run

    def gather(self, C, ldc, I, J):
        """Entries C[I[s], J[s]] of a device matrix (row stride ldc) on the host."""
        idx = self.torch.from_numpy(np.asarray(I, np.int64) * ldc + np.asarray(J, np.int64)).to(self.dev)
        return C.reshape(-1)[idx].cpu().numpy().astype(np.float64)


# ============================================================ oracle leg ===
# The only code in this file that calls the oracle: CPU work after the GPU
# timing, scoring GPU results and timing the oracle itself.

def oracle_error(tA, tB, m, n, k, alpha, A_h, lda, B_h, ldb, beta, C0_h, got, I, J):
    """Normalised error of GPU values `got` at (I, J) against the oracle."""
    import oracle
    cref, d = oracle.gemm_entries(tA, tB, k, alpha, A_h, lda, B_h, ldb, beta, C0_h, n, I, J)
    return float(f"{oracle.normalized_error(got, cref, d):.3e}")


def cpu_baseline(A_h, B_h, C0_h, gpu_rows, target_s=25.0):
    """Time the FP64 oracle on a block of output rows of the 8192^3 GEMM on
    every host core, and score the GPU results on those rows."""
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
    errs = {p: float(f"{oracle.normalized_error(g[:rows].astype(np.float64), Cref, D):.3e}")
            for p, g in gpu_rows.items()}
    return {"value": 2.0 * rows * N * K / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {rows} of {M} output rows of the same 8192^3 GEMM "
                      f"({rows * N} outputs, full K), FP64 triple loop, {dt:.1f} s"}, errs


def oracle_config1(a, b, c_gpu):
    """The small workload (256^3 NN, alpha 1, beta 0) on the oracle: its time
    on one thread (the paper's single-thread setting, Section 4.1.3) and on
    every host core, and the GPU result's error over all 65536 outputs."""
    import oracle
    n = 256
    out = {}
    for name, threads in (("one_thread", 1), ("all_cores", oracle.max_threads())):
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            ref, d = oracle.gemm("N", "N", n, n, n, 1.0, a, n, b, n, 0.0, None, n, threads=threads)
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        out[name] = {"threads": threads, "ms": round(t * 1e3, 3), "gflops": round(2.0 * n ** 3 / t / 1e9, 3)}
    out["gpu_error_vs_fp64_oracle_all_outputs"] = float(f"{oracle.normalized_error(c_gpu, ref, d):.3e}")
    return out


def oracle_chain_errors(X, W1, W2, G, Y, grads):
    """Sampled oracle values of Y and the three gradients (16 x 16 entries each,
    chained denominators)."""
    import oracle
    out = {}
    for name, (I, J, ref, den) in oracle.chain_entries(X, W1, W2, G).items():
        got = Y[np.ix_(I, J)] if name == "Y" else grads[name][np.ix_(I, J)]
        out[name] = float(f"{oracle.normalized_error(got.astype(np.float64), ref, den):.3e}")
    return out


def oracle_syr2k_error(trans, k, alpha, X_h, Y_h, ld, beta, C0_h, n, got, I, J):
    import oracle
    ref, d = oracle.syr2k_entries(trans, k, alpha, X_h, ld, Y_h, ld, beta, C0_h, n, I, J)
    return float(f"{oracle.normalized_error(got, ref, d):.3e}")


def oracle_i8_mismatches(a, b, alpha, got, I, J):
    """Sampled INT8 outputs (beta 0) that differ from the exact integer oracle."""
    import oracle
    k = a.shape[1]
    want = np.array([oracle.gemm_i8("N", "N", 1, 1, k, alpha, a[i], k, np.ascontiguousarray(b[:, j]), 1)[0, 0]
                     for i, j in zip(I, J)], dtype=np.int64)
    return int(np.count_nonzero(np.asarray(got, np.int64) != want))


# ============================================================= workloads ===

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=3,
                    help="rounds of shuffled cases (multi-case workloads)")
    ap.add_argument("--order-seed", type=int, default=None,
                    help="seed of the case-order shuffle (default: drawn at random and reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["sgemm", "batched", "chain", "mixed", "fp8", "sweep", "tiling",
                                           "engine", "types", "syr2k", "smallk"],
                    default="sgemm",
                    help="sgemm: the FP32 8192^3 line (default); batched: 512 uneven problems; "
                         "chain: forward + backward of Y = (X W1) W2; mixed (alias fp8): bf16x3, BF16, FP16 "
                         "and FP8 at 8192^3 on both input distributions; sweep: FP32 shapes x layouts; "
                         "tiling: Tiling vs Tiling+Packing over sizes; engine: vector-ALU vs matrix-core "
                         "micro-kernel; types: FP16 and INT8 at 8192^3; syr2k: SYR2K at N = K = 8192; "
                         "smallk: 8192 x 8192 x 256 with warm and flushed caches")
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
    _native.lib()
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    bench = Bench(args, torch, _native, dev)
    progress(f"workload {args.workload}, order seed {bench.order_seed}")
    fn = {"sgemm": bench_sgemm, "batched": bench_batched, "chain": bench_chain, "mixed": bench_mixed,
          "fp8": bench_mixed, "sweep": bench_sweep, "tiling": bench_tiling, "engine": bench_engine,
          "types": bench_types, "syr2k": bench_syr2k, "smallk": bench_smallk}[args.workload]
    out = fn(bench, si)
    out["order_seed"] = bench.order_seed
    print(json.dumps(out), flush=True)


def header(bench, metric, unit, value, ms, dtype, config, higher=True):
    a = bench.args
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def bench_sgemm(bench, si):
    torch, dev, args = bench.torch, bench.dev, bench.args
    A_h = si.uniform((M, K), si.seed_for(2, "A")).reshape(-1)
    B_h = si.uniform((K, N), si.seed_for(2, "B")).reshape(-1)
    C0_h = si.uniform((M, N), si.seed_for(2, "C")).reshape(-1)
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    C0 = torch.from_numpy(C0_h).to(dev)

    flops = 2.0 * M * N * K
    order = bench.shuffled(["fp32", "bf16x3"])
    res = {}
    for path in order:
        C = C0.clone()
        run = bench.gemm_call(path, "N", "N", M, N, K, ALPHA, A, K, B, N, BETA, C, N)
        res[path] = bench.case(run)
        del C, run
    f32 = res["fp32"]
    f32_cfg = native_plan_config(bench, M, N, K)
    ms = f32["total_ms"] / args.steps
    achieved = tflops(flops, float(np.mean(f32["per_ms"])))
    peak = PEAK_TFLOPS["fp32"]
    out = header(bench, METRIC, "TFLOP/s", round(tflops(flops, ms), 2), round(ms, 4), "f32",
                 {"workload": "sgemm_fp32_8192x8192x8192_nn", "M": M, "N": N, "K": K, "layout": "NN",
                  "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]", "path": "fp32"})
    out["pct_fp32_mfma_peak"] = round(100.0 * tflops(flops, ms) / peak, 2)
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                       "frac": round(achieved / peak, 4), "traffic": measured_traffic(),
                       "kernel": "sgemm_mfma_kernel<256,256,16,128,64,NN> (configuration %d%s)" % (
                           f32_cfg, ", two register staging sets" if f32_cfg == 17 else ""),
                       "kernel_ms_mean": round(float(np.mean(f32["per_ms"])), 4),
                       "algorithmic_flops_per_launch": flops}
    out["step_time_ms"] = {p: stats(r["per_ms"]) for p, r in res.items()}
    out["sclk_mhz"] = {p: r["sclk_mhz"] for p, r in res.items()}
    out["sclk_mhz_during"] = {p: r["sclk_mhz_during"] for p, r in res.items()}
    if f32["sclk_mhz"]:
        out["pct_fp32_mfma_peak_at_measured_clock"] = round(
            100.0 * tflops(flops, ms) / (peak * f32["sclk_mhz"] / 2400.0), 2)
    out["order"] = order
    b = res["bf16x3"]
    bms = b["total_ms"] / args.steps
    out["bf16x3"] = {"tflops": round(tflops(flops, bms), 2), "ms_per_step": round(bms, 4),
                     "speedup_vs_fp32": round(ms / bms, 3),
                     "pct_bf16_mfma_peak_issued": round(100.0 * 3 * tflops(flops, bms) / PEAK_TFLOPS["bf16"], 2)}
    # one GEMM per path from the original C0, for the error check
    outs = {}
    rows_needed = 512
    for path in res:
        C = C0.clone()
        bench.gemm_call(path, "N", "N", M, N, K, ALPHA, A, K, B, N, BETA, C, N)()
        torch.cuda.synchronize()
        outs[path] = C[: rows_needed * N].cpu().numpy().reshape(rows_needed, N)
        del C
    # the small workload (256^3 NN, alpha 1, beta 0): GPU time per launch
    n1 = 256
    a1 = si.uniform((n1, n1), si.seed_for(1, "A"))
    b1 = si.uniform((n1, n1), si.seed_for(1, "B"))
    dA1, dB1 = torch.from_numpy(a1).to(dev), torch.from_numpy(b1).to(dev)
    dC1 = torch.zeros((n1, n1), device=dev)
    run1 = bench.gemm_call("fp32", "N", "N", n1, n1, n1, 1.0, dA1, n1, dB1, n1, 0.0, dC1, n1)
    bench.warm(run1, args.warmup)
    t1 = bench.per_launch(run1, max(args.steps, 50))
    c1 = dC1.cpu().numpy().astype(np.float64)

    # ---- oracle leg
    progress("GPU timing done; oracle leg")
    if not args.no_cpu_baseline:
        cb, errs = cpu_baseline(A_h, B_h, C0_h, outs)
        out["cpu_baseline"] = cb
        out["sampled_error_vs_fp64_oracle"] = errs
        out["error_sample"] = "the cpu_baseline's block of output rows (every output in them)"
    else:
        I, J = si.sample_indices(rows_needed, N, SAMPLES, 301)
        out["cpu_baseline"] = None
        out["sampled_error_vs_fp64_oracle"] = {
            p: oracle_error("N", "N", M, N, K, ALPHA, A_h, K, B_h, N, BETA, C0_h, g[I, J].astype(np.float64), I, J)
            for p, g in outs.items()}
        out["error_sample"] = f"{len(I)} outputs of the first {rows_needed} rows"
    cfg1 = {"workload": "sgemm_fp32_256x256x256_nn",
            "gpu_us_per_launch_median": round(float(np.median(t1)) * 1e3, 2)}
    cfg1.update(oracle_config1(a1, b1, c1))
    out["small_workload_256"] = cfg1
    return out


SWEEP_SHAPES = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
                (8192, 8192, 256), (256, 8192, 8192), (16384, 1024, 4096),
                # shapes whose workgroups do not fall into whole rounds over the
                # compute units (the FP32 round plan and the 16-bit split rule)
                (1536, 1536, 1536), (3072, 3072, 3072), (6144, 6144, 6144), (3072, 3072, 1024)]


def bench_sweep(bench, si):
    """The FP32 sweep (alpha 1.5, beta 0.5, U[-1, 1]) in all four layouts on the
    FP32 path and NN on the bf16x3 path.  Every round runs every case once, in
    a freshly shuffled order; per case: the median and CI of all its steps,
    the clock after each of its blocks, and the sampled oracle error of one
    GEMM from the original C0."""
    torch, dev, args = bench.torch, bench.dev, bench.args
    data = {}
    for (m, n, k) in SWEEP_SHAPES:
        A_h = si.uniform((m * k,), si.seed_for(2, "A"))
        B_h = si.uniform((k * n,), si.seed_for(2, "B"))
        C0_h = si.uniform((m * n,), si.seed_for(2, "C"))
        data[(m, n, k)] = (A_h, B_h, C0_h, torch.from_numpy(A_h).to(dev), torch.from_numpy(B_h).to(dev),
                           torch.from_numpy(C0_h).to(dev), torch.from_numpy(C0_h).to(dev))
    cases = [("fp32", s, tA + tB) for s in SWEEP_SHAPES for tA in "NT" for tB in "NT"]
    cases += [("bf16x3", s, "NN") for s in SWEEP_SHAPES]
    runs, samples, clocks, calls = {}, {c: [] for c in cases}, {c: [] for c in cases}, {}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for case in bench.shuffled(cases):
            path, (m, n, k), lay = case
            A_h, B_h, C0_h, A, B, C0, C = data[(m, n, k)]
            lda = k if lay[0] == "N" else m
            ldb = n if lay[1] == "N" else k
            if case not in runs:
                runs[case] = bench.gemm_call(path, lay[0], lay[1], m, n, k, ALPHA, A, lda, B, ldb, BETA, C, n)
            r = bench.case(runs[case])
            samples[case] += r["per_ms"]
            clocks[case].append([r["sclk_mhz_during"], r["sclk_mhz"]])
            calls[case] = r["calls_per_sample"]
    rows = []
    for case in cases:
        path, (m, n, k), lay = case
        A_h, B_h, C0_h, A, B, C0, C = data[(m, n, k)]
        lda = k if lay[0] == "N" else m
        ldb = n if lay[1] == "N" else k
        Cf = C0.clone()
        bench.gemm_call(path, lay[0], lay[1], m, n, k, ALPHA, A, lda, B, ldb, BETA, Cf, n,
                        ws=runs[case].workspace)()
        I, J = si.sample_indices(m, n, SAMPLES, 302)
        got = bench.gather(Cf, n, I, J)
        del Cf
        flops = 2.0 * m * n * k
        ms = float(np.mean(samples[case]))
        st, cfg, splits, packed = bench.native.mg_gemm_plan(PATH_ID[path], m, n, k,
                                                            runs[case].workspace.numel())
        rows.append({"M": m, "N": n, "K": k, "path": path, "layout": lay, "ms": round(ms, 5),
                     "tflops": round(tflops(flops, ms), 2),
                     "pct_fp32_peak": round(100 * tflops(flops, ms) / PEAK_TFLOPS["fp32"], 1),
                     "step_ms": stats(samples[case]), "calls_per_sample": calls[case], "sclk_mhz": clocks[case],
                     "config": cfg, "splits": splits, "prepacked": packed,
                     "sampled_error_vs_fp64_oracle": oracle_error(lay[0], lay[1], m, n, k, ALPHA, A_h, lda, B_h, ldb,
                                                                  BETA, C0_h, got, I, J)})
    nn8 = [r for r in rows if r["M"] == 8192 and r["K"] == 8192 and r["path"] == "fp32" and r["layout"] == "NN"][0]
    out = header(bench, "FP32 SGEMM sweep TFLOP/s (all layouts) and bf16x3 NN", "TFLOP/s", nn8["tflops"],
                 nn8["ms"], "f32", {"workload": "sgemm_sweep", "alpha": ALPHA, "beta": BETA,
                                    "inputs": "uniform[-1,1]", "rounds": args.rounds})
    out["rows"] = rows
    out["worst_error"] = {p: max(r["sampled_error_vs_fp64_oracle"] for r in rows if r["path"] == p)
                          for p in ("fp32", "bf16x3")}
    return out


def bench_mixed(bench, si):
    """The mixed-precision workload at 8192^3 (NN, alpha 1, beta 0): bf16x3,
    BF16, FP16 and FP8 (E4M3, per-128x128-tile scales) on FP32 inputs drawn
    uniform[-1, 1] and log-uniform in magnitude over [1e-3, 1e3] with random
    sign.  Every path is timed end to end from FP32 operands; FP8 also GEMM
    only (operands packed once) and the pack alone.  Cases run in shuffled
    order per round; each reports the oracle error of its output."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    sp = bench.sp
    gens = {"uniform": si.uniform, "log": si.log_uniform_signed}
    host, devm = {}, {}
    for dist, gen in gens.items():
        host[dist] = (gen((M, K), si.seed_for(3, "A")), gen((K, N), si.seed_for(3, "B")))
        devm[dist] = tuple(torch.from_numpy(x.reshape(-1)).to(dev) for x in host[dist])
    C = torch.zeros(M * N, device=dev)
    qa_b, sa_b = native.mg_fp8_packed_size(M, K)
    qb_b, sb_b = native.mg_fp8_packed_size(N, K)
    packs = {dist: tuple(torch.empty(x, dtype=torch.uint8, device=dev) for x in (qa_b, sa_b, qb_b, sb_b))
             for dist in gens}

    def pack_fn(dist):
        A, B = devm[dist]
        qA, sA, qB, sB = packs[dist]

        def pack():
            native.check(native.mg_fp8_pack("N", M, K, A.data_ptr(), K, qA.data_ptr(), sA.data_ptr(), sp), "pack A")
            native.check(native.mg_fp8_pack("T", N, K, B.data_ptr(), N, qB.data_ptr(), sB.data_ptr(), sp), "pack B")
        return pack

    def gemm_only_fn(dist, Cd):
        qA, sA, qB, sB = packs[dist]
        return lambda: native.check(native.mg_gemm_fp8_packed(M, N, K, 1.0, qA.data_ptr(), sA.data_ptr(),
                                                              qB.data_ptr(), sB.data_ptr(), 0.0, Cd.data_ptr(), N,
                                                              sp), "fp8 gemm")

    paths = ["bf16x3", "bf16", "fp16", "fp8"]
    kinds = paths + ["fp8_gemm_only", "fp8_pack"]
    cases = [(d, p) for d in gens for p in kinds]
    for dist in gens:
        pack_fn(dist)()
    torch.cuda.synchronize()
    runs, per, clk = {}, {c: [] for c in cases}, {c: [] for c in cases}
    ws = None
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for case in bench.shuffled(cases):
            dist, p = case
            if case not in runs:
                A, B = devm[dist]
                if p == "fp8_pack":
                    runs[case] = pack_fn(dist)
                elif p == "fp8_gemm_only":
                    runs[case] = gemm_only_fn(dist, C)
                else:
                    runs[case] = bench.gemm_call(p, "N", "N", M, N, K, 1.0, A, K, B, N, 0.0, C, N, ws=ws)
                    ws = runs[case].workspace
            r = bench.case(runs[case])
            per[case] += r["per_ms"]
            clk[case].append([r["sclk_mhz_during"], r["sclk_mhz"]])
    flops = 2.0 * M * N * K
    I, J = si.sample_indices(M, N, SAMPLES, 303)
    rows = {}
    for dist in gens:
        a_h, b_h = host[dist]
        rows[dist] = {}
        for p in kinds:
            ms = float(np.mean(per[(dist, p)]))
            row = {"ms": round(ms, 5), "step_ms": stats(per[(dist, p)]), "sclk_mhz": clk[(dist, p)]}
            if p == "fp8_pack":
                row["gbps"] = round(2 * (4.0 + 1.0) * M * K / (ms * 1e-3) / 1e9, 1)
                rows[dist][p] = row
                continue
            base = "fp8" if p.startswith("fp8") else p
            row["tflops"] = round(tflops(flops, ms), 2)
            row["pct_dtype_peak_issued"] = round(100 * ISSUED[base] * tflops(flops, ms) / DTYPE_PEAK[base], 2)
            Cf = torch.zeros(M * N, device=dev)
            if p == "fp8_gemm_only":
                gemm_only_fn(dist, Cf)()
            else:
                A, B = devm[dist]
                bench.gemm_call(p, "N", "N", M, N, K, 1.0, A, K, B, N, 0.0, Cf, N, ws=ws)()
            got = bench.gather(Cf, N, I, J)
            del Cf
            row["sampled_error_vs_fp64_oracle"] = oracle_error("N", "N", M, N, K, 1.0, a_h, K, b_h, N, 0.0, None,
                                                               got, I, J)
            row["tolerance"] = TOL[base]
            rows[dist][p] = row
    u = rows["uniform"]
    out = header(bench, "Mixed-precision GEMM TFLOP/s at 8192^3 (bf16x3, BF16, FP16, FP8 per-tile scales), "
                        "error vs FP64 oracle per variant and input distribution", "TFLOP/s",
                 u["fp8"]["tflops"], u["fp8"]["ms"], "fp8_e4m3",
                 {"workload": "gemm_mixed_precision_8192x8192x8192_nn", "M": M, "N": N, "K": K, "layout": "NN",
                  "alpha": 1.0, "beta": 0.0,
                  "inputs": {"uniform": "uniform[-1,1]", "log": "|x| = 10^U(-3,3), random sign"},
                  "rounds": args.rounds})
    fo = u["fp8_gemm_only"]
    out["roofline"] = {"bound": "mfma", "achieved": fo["tflops"], "peak": PEAK_TFLOPS["fp8"], "unit": "TFLOP/s",
                       "frac": round(fo["tflops"] / PEAK_TFLOPS["fp8"], 4), "traffic": None,
                       "kernel": tuned_kernel_name(bench.native, 3, "gemm_fp8_direct_kernel", M, N, K)
                       + ", FP8 GEMM on packed operands",
                       "kernel_ms_mean": fo["ms"], "algorithmic_flops_per_launch": flops}
    out["rows"] = rows
    return out


def bench_batched(bench, si):
    """512 GEMMs with M, N, K log-uniform in [32, 2048] (multiples of 8),
    U[-1, 1], alpha 1, beta 0: one persistent launch, against one launch per
    problem (the device time of the 512 launches replayed from one HIP graph,
    and the wall time of the host loop that issues them one by one)."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    sp = bench.sp
    sizes = si.batched_sizes(512, si.seed_for(4, "A"))
    host, ops = [], []
    for i, (m, n, k) in enumerate(sizes):
        a = si.uniform((m, k), si.seed_for(4, "A", i))
        b = si.uniform((k, n), si.seed_for(4, "B", i))
        host.append((a, b))
        ops.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), torch.zeros((m, n), device=dev)))
    flops = sum(2.0 * m * n * k for m, n, k in sizes)
    out = header(bench, "uneven batched GEMM TFLOP/s, 512 problems in one persistent launch", "TFLOP/s", None,
                 None, "f32", {"workload": "batched_uneven_512", "problems": 512,
                               "sizes": "M,N,K log-uniform in [32, 2048], multiples of 8", "layout": "NN",
                               "alpha": 1.0, "beta": 0.0, "total_gflop": round(flops / 1e9, 2),
                               "rounds": args.rounds})
    out["paths"] = {}
    arrs, wss = {}, {}
    for path in ("fp32", "bf16x3"):
        pid = PATH_ID[path]
        arr = (native.mg_problem * len(ops))()
        for i, (A, B, C) in enumerate(ops):
            m, k = A.shape
            n = B.shape[1]
            arr[i] = native.mg_problem(b"N", b"N", m, n, k, 1.0, 0.0, A.data_ptr(), k, B.data_ptr(), n,
                                       C.data_ptr(), n)
        arrs[path] = arr
        need = native.mg_gemm_batched_workspace_size(pid, len(ops))
        wss[path] = (torch.empty(need, dtype=torch.uint8, device=dev), need)

    def persistent(path):
        pid, arr, (ws, need) = PATH_ID[path], arrs[path], wss[path]
        return lambda: native.check(native.mg_gemm_batched(pid, len(ops), arr, ws.data_ptr(), need, sp)[0],
                                    "mg_gemm_batched")

    single = {}

    def one(path, i):
        if (path, i) not in single:
            A, B, C = ops[i]
            m, k = A.shape
            n = B.shape[1]
            single[(path, i)] = bench.gemm_call(path, "N", "N", m, n, k, 1.0, A, k, B, n, 0.0, C, n)
        return single[(path, i)]

    def loop(path):
        fns = [one(path, i) for i in range(len(ops))]

        def run():
            for f in fns:
                f()
        return run

    cases = [(p, kind) for p in ("fp32", "bf16x3") for kind in ("persistent", "host_loop")]
    per = {c: [] for c in cases}
    clk = {c: [] for c in cases}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for case in bench.shuffled(cases):
            path, kind = case
            r = bench.case(persistent(path) if kind == "persistent" else loop(path))
            per[case] += r["per_ms"]
            clk[case].append([r["sclk_mhz_during"], r["sclk_mhz"]])
    for path in ("fp32", "bf16x3"):
        dms, graph_ok = _per_problem_graph(bench, path, ops, one)
        pms = float(np.mean(per[(path, "persistent")]))
        lms = float(np.mean(per[(path, "host_loop")]))
        res = {"persistent": {"ms": round(pms, 4), "tflops": round(tflops(flops, pms), 2), "launches": 1,
                              "step_ms": stats(per[(path, "persistent")]), "sclk_mhz": clk[(path, "persistent")]},
               "per_problem_device": {"ms": round(dms, 4), "tflops": round(tflops(flops, dms), 2),
                                      "launches": len(ops), "replays_match_eager": graph_ok,
                                      "how": "the 512 single-GEMM launches captured in one HIP graph and "
                                             "replayed (device time without the host's per-call overhead)"},
               "per_problem_host_loop": {"ms": round(lms, 4), "tflops": round(tflops(flops, lms), 2),
                                         "launches": len(ops), "step_ms": stats(per[(path, "host_loop")])},
               "speedup_vs_per_problem_device": round(dms / pms, 3),
               "speedup_vs_host_loop": round(lms / pms, 3)}
        res["persistent"].update(_batched_tail(bench, PATH_ID[path], arrs[path], len(ops), *wss[path]))
        # error: one persistent launch into zeroed outputs, 64 sampled outputs per problem
        for _, _, C in ops:
            C.zero_()
        persistent(path)()
        torch.cuda.synchronize()
        worst = 0.0
        for i, ((a, b), (_, _, C)) in enumerate(zip(host, ops)):
            m, n = C.shape
            I, J = si.sample_indices(m, n, 64, 400 + i)
            got = bench.gather(C, n, I, J)
            worst = max(worst, oracle_error("N", "N", m, n, a.shape[1], 1.0, a, a.shape[1], b, n, 0.0, None,
                                            got, I, J))
        res["sampled_error_vs_fp64_oracle_worst_problem"] = worst
        out["paths"][path] = res
    out["value"] = out["paths"]["fp32"]["persistent"]["tflops"]
    out["ms_per_step"] = out["paths"]["fp32"]["persistent"]["ms"]
    out["bf16x3_vs_fp32_persistent"] = round(out["paths"]["bf16x3"]["persistent"]["tflops"] / out["value"], 3)
    return out


def _per_problem_graph(bench, path, ops, one):
    """Median time of one replay of a HIP graph holding the 512 per-problem
    mg_gemm launches (their workspaces allocated before capture), and whether
    every replay reproduced the eager launches' outputs bit for bit."""
    torch, native = bench.torch, bench.native
    runs = [one(path, i) for i in range(len(ops))]          # allocates the workspaces
    for r in runs:
        r()
    torch.cuda.synchronize()
    eager = [C.clone() for _, _, C in ops]
    pid = PATH_ID[path]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cs = torch.cuda.current_stream().cuda_stream
        for (A, B, C), r in zip(ops, runs):
            m, k = A.shape
            n = B.shape[1]
            ws = r.workspace
            need = native.mg_gemm_workspace_size(pid, "N", "N", m, n, k)
            native.check(native.mg_gemm(pid, "N", "N", m, n, k, 1.0, A.data_ptr(), k, B.data_ptr(), n, 0.0,
                                        C.data_ptr(), n, ws.data_ptr(), need, cs), "mg_gemm (capture)")
    ok = True
    times = []
    for rep in range(6):
        for _, _, C in ops:
            C.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bench.stream)
        g.replay()
        e1.record(bench.stream)
        torch.cuda.synchronize()
        if rep:
            times.append(e0.elapsed_time(e1))
        ok = ok and all(torch.equal(C, E) for (_, _, C), E in zip(ops, eager))
    del g
    return float(np.median(times)), ok


def _batched_tail(bench, pid, arr, count, ws, need):
    """One more persistent launch with per-workgroup wall-clock stamps: how
    long the workgroups that found the work list empty waited for the last
    tiles.  tail_idle_frac = sum over workgroups of (last end - own end) over
    workgroups x (last end - first start)."""
    torch, native = bench.torch, bench.native
    slots = native.mg_batched_slots(pid)
    stamps = torch.zeros(2 * slots, dtype=torch.int64, device=bench.dev)
    st, bad, grid = native.mg_gemm_batched_timed(pid, count, arr, ws.data_ptr(), need, bench.sp,
                                                 stamps.data_ptr(), 2 * slots)
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


def bench_chain(bench, si):
    """Y = (X W1) W2 with X 4096x2048, W1 2048x8192, W2 8192x2048; one step is
    the forward (2 GEMMs) and the hand-written backward (4 GEMMs) of
    loss = sum(Y * G), on the bf16x3 path and on the FP32 path (shuffled per
    round).  Errors: Y and dX, dW1, dW2 at 16 x 16 sampled entries each
    against the FP64 oracle with chained denominators."""
    torch, dev, args = bench.torch, bench.dev, bench.args
    from paper_2305_18236_amd.autograd import chain
    Mx, D, Hd = 4096, 2048, 8192
    h = {"X": si.uniform((Mx, D), si.seed_for(5, "X")), "W1": si.uniform((D, Hd), si.seed_for(5, "W1")),
         "W2": si.uniform((Hd, D), si.seed_for(5, "W2")), "G": si.gaussian((Mx, D), si.seed_for(5, "G"))}
    X = torch.from_numpy(h["X"]).to(dev).requires_grad_(True)
    W1 = torch.from_numpy(h["W1"]).to(dev).requires_grad_(True)
    W2 = torch.from_numpy(h["W2"]).to(dev).requires_grad_(True)
    G = torch.from_numpy(h["G"]).to(dev)
    flops = 6 * 2.0 * Mx * D * Hd
    out = header(bench, "differentiable GEMM chain TFLOP/s (forward + hand-written backward)", "TFLOP/s", None,
                 None, "bf16x3", {"workload": "gemm_chain_4096x2048x8192", "X": [Mx, D], "W1": [D, Hd],
                                  "W2": [Hd, D], "loss": "sum(Y*G), G ~ N(0,1)", "gemms_per_step": 6,
                                  "gflop_per_step": round(flops / 1e9, 1), "rounds": args.rounds})
    last = {}

    def step_fn(path):
        def step():
            for t in (X, W1, W2):
                t.grad = None
            Y = chain(X, W1, W2, path)
            Y.backward(G)
            last[path] = Y
        return step

    per = {p: [] for p in ("bf16x3", "fp32")}
    clk = {p: [] for p in per}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for path in bench.shuffled(per):
            r = bench.case(step_fn(path))
            per[path] += r["per_ms"]
            clk[path].append([r["sclk_mhz_during"], r["sclk_mhz"]])
    out["paths"] = {}
    for path in per:
        step_fn(path)()
        torch.cuda.synchronize()
        grads = {"dX": X.grad.cpu().numpy(), "dW1": W1.grad.cpu().numpy(), "dW2": W2.grad.cpu().numpy()}
        Y = last[path].detach().cpu().numpy()
        ms = float(np.mean(per[path]))
        out["paths"][path] = {"ms_per_step": round(ms, 4), "tflops": round(tflops(flops, ms), 2),
                              "step_ms": stats(per[path]), "sclk_mhz": clk[path],
                              "sampled_error_vs_fp64_oracle": oracle_chain_errors(h["X"], h["W1"], h["W2"], h["G"],
                                                                                  Y, grads),
                              "tolerance": 2e-5}
    b, f = out["paths"]["bf16x3"], out["paths"]["fp32"]
    out["value"] = b["tflops"]
    out["ms_per_step"] = b["ms_per_step"]
    out["speedup_bf16x3_vs_fp32"] = round(f["ms_per_step"] / b["ms_per_step"], 3)
    return out


TILING_SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]


def bench_tiling(bench, si):
    """The packing ablation of the paper's Section 4.1.3 on the FP32 path:
    square SGEMMs C = A B (NN, alpha 1, beta 0) over the paper's sizes, each
    timed with every tile configuration; "Tiling" is the best configuration
    that loads operands straight into registers, "Tiling+Packing" the best one
    that packs them into LDS (split-K allowed for both, as the library would
    run them).  Configurations run in shuffled order per size; each best
    configuration's output is scored against the oracle."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    ncfg = native.mg_num_configs(0)
    rows = []
    for n in TILING_SIZES:
        progress(f"size {n}")
        a = si.uniform((n * n,), si.seed_for(2, "A"))
        b = si.uniform((n * n,), si.seed_for(2, "B"))
        A, B = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
        C = torch.zeros(n * n, device=dev)
        steps = max(args.steps, 200 if n <= 512 else 20)
        I, J = si.sample_indices(n, n, SAMPLES, 304)
        per_cfg, clocks, outs = {}, {}, {}
        for cfg in bench.shuffled(range(ncfg)):
            native.check(native.mg_force_config(0, cfg), "mg_force_config")
            try:
                run = bench.gemm_call("fp32", "N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)
                bench.warm(run, args.warmup)
                per_cfg[cfg] = float(np.median(bench.per_launch(run, steps)))
                clocks[cfg] = bench.sclk()
                outs[cfg] = bench.gather(C, n, I, J)
            finally:
                native.mg_force_config(0, -1)
        flops = 2.0 * n ** 3
        best = {}
        for name, packs in (("tiling", 0), ("tiling_packing", 1)):
            cands = {c: t for c, t in per_cfg.items() if native.mg_config_packs(0, c) == packs}
            c = min(cands, key=cands.get)
            best[name] = {"config": c, "us": round(cands[c] * 1e3, 2),
                          "tflops": round(tflops(flops, cands[c]), 3), "sclk_mhz": clocks[c],
                          "sampled_error_vs_fp64_oracle": oracle_error("N", "N", n, n, n, 1.0, a, n, b, n, 0.0,
                                                                       None, outs[c], I, J)}
        rows.append({"M": n, "N": n, "K": n, **best,
                     "packing_speedup": round(best["tiling"]["us"] / best["tiling_packing"]["us"], 3),
                     "auto_config": native.mg_tuned_config(0, n, n, n)})
        del A, B, C
    big = rows[-1]
    out = header(bench, "FP32 SGEMM time, Tiling vs Tiling+Packing over sizes", "TFLOP/s",
                 big["tiling_packing"]["tflops"], big["tiling_packing"]["us"] / 1e3, "f32",
                 {"workload": "sgemm_packing_ablation", "alpha": 1.0, "beta": 0.0, "layout": "NN",
                  "inputs": "uniform[-1,1]", "timing": "median over launches of HIP events recorded around each call"})
    out["rows"] = rows
    return out


ENGINE_SIZES = [1024, 2048, 4096, 8192]
# FP32 on the vector ALUs: the published 157.3 TFLOP/s (256 flop per clock per
# CU at 2.4 GHz).  The kernels issue scalar v_fmac_f32 only (packed FP32 is
# disabled at build time); they measure above 78.6 TFLOP/s, so scalar FMAs are
# not limited to half the vector rate on this chip and the full figure is the
# bound.
VALU_FP32_PEAK = 256 * 256 * 2.4e9 / 1e12


def bench_engine(bench, si):
    """The paper's generic-vs-MMA lowering comparison (Section 4.4) on the GPU:
    the same packed macro level with the vector-ALU FMA micro-kernel and with
    the MFMA micro-kernel, square FP32 SGEMMs (NN, alpha 1.5, beta 0.5).  MFMA
    runs the automatic configuration; VALU the best of its configurations."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    ncfg = native.mg_num_configs(0)
    valu_cfgs = [c for c in range(ncfg) if native.mg_config_uses_mfma(0, c) == 0]
    rows = []
    for n in ENGINE_SIZES:
        progress(f"size {n}")
        a = si.uniform((n * n,), si.seed_for(2, "A"))
        b = si.uniform((n * n,), si.seed_for(2, "B"))
        c0 = si.uniform((n * n,), si.seed_for(2, "C"))
        A, B, C0 = (torch.from_numpy(x).to(dev) for x in (a, b, c0))
        C = C0.clone()
        steps = args.steps if n >= 4096 else max(args.steps, 50)
        I, J = si.sample_indices(n, n, SAMPLES, 305)

        def timed(cfg):
            if cfg is not None:
                native.check(native.mg_force_config(0, cfg), "mg_force_config")
            try:
                run = bench.gemm_call("fp32", "N", "N", n, n, n, ALPHA, A, n, B, n, BETA, C, n)
                r = bench.case(run, steps=steps)
                Cf = C0.clone()
                bench.gemm_call("fp32", "N", "N", n, n, n, ALPHA, A, n, B, n, BETA, Cf, n, ws=run.workspace)()
                got = bench.gather(Cf, n, I, J)
                return float(np.mean(r["per_ms"])), r["sclk_mhz"], got
            finally:
                native.mg_force_config(0, -1)

        res = {}
        for c in bench.shuffled(valu_cfgs + [None]):
            res[c] = timed(c)
        mfma_ms, mfma_clk, mfma_got = res.pop(None)
        vc = min(res, key=lambda c: res[c][0])
        flops = 2.0 * n ** 3
        tf_v, tf_m = tflops(flops, res[vc][0]), tflops(flops, mfma_ms)
        rows.append({"M": n, "N": n, "K": n,
                     "valu": {"config": vc, "ms": round(res[vc][0], 4), "tflops": round(tf_v, 2),
                              "frac_of_valu_peak": round(tf_v / VALU_FP32_PEAK, 3), "sclk_mhz": res[vc][1],
                              "sampled_error_vs_fp64_oracle": oracle_error("N", "N", n, n, n, ALPHA, a, n, b, n, BETA,
                                                                           c0, res[vc][2], I, J)},
                     "mfma": {"config": native.mg_tuned_config(0, n, n, n), "ms": round(mfma_ms, 4),
                              "tflops": round(tf_m, 2), "frac_of_mfma_peak": round(tf_m / PEAK_TFLOPS["fp32"], 3),
                              "sclk_mhz": mfma_clk,
                              "sampled_error_vs_fp64_oracle": oracle_error("N", "N", n, n, n, ALPHA, a, n, b, n, BETA,
                                                                           c0, mfma_got, I, J)},
                     "mfma_speedup": round(res[vc][0] / mfma_ms, 3)})
        del A, B, C, C0
    big = rows[-1]
    out = header(bench, "FP32 SGEMM TFLOP/s, vector-ALU vs matrix-core micro-kernel", "TFLOP/s",
                 big["valu"]["tflops"], big["valu"]["ms"], "f32",
                 {"workload": "sgemm_valu_vs_mfma", "alpha": ALPHA, "beta": BETA, "layout": "NN",
                  "inputs": "uniform[-1,1]"})
    out["roofline"] = {"bound": "alu", "achieved": big["valu"]["tflops"], "peak": round(VALU_FP32_PEAK, 1),
                       "unit": "TFLOP/s", "frac": big["valu"]["frac_of_valu_peak"], "traffic": None,
                       "kernel": f"sgemm_valu_kernel (config {big['valu']['config']}) at 8192^3"}
    out["rows"] = rows
    return out


INT8_PEAK_TOPS = 5033.2


def bench_types(bench, si):
    """Table 1's other operand types at 8192^3 NN: the FP16 path (FP32
    operands rounded to binary16, end to end) and the INT8 entry points (int8
    operands, int32 C; end to end including the pack, and the GEMM alone on
    packed operands).  alpha 1, beta 0.  Cases run in shuffled order per
    round; FP16 is scored against the FP64 oracle, INT8 against the exact
    integer oracle."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    sp = bench.sp
    n = M
    flops = 2.0 * n ** 3
    a16, b16 = si.uniform((n * n,), si.seed_for(3, "A")), si.uniform((n * n,), si.seed_for(3, "B"))
    A, B = torch.from_numpy(a16).to(dev), torch.from_numpy(b16).to(dev)
    C = torch.zeros(n * n, device=dev)
    rng = np.random.default_rng(si.seed_for(3, "X"))
    a8 = rng.integers(-128, 128, (n, n), dtype=np.int8)
    b8 = rng.integers(-128, 128, (n, n), dtype=np.int8)
    Ai, Bi = torch.from_numpy(a8).to(dev), torch.from_numpy(b8).to(dev)
    Ci = torch.zeros(n * n, dtype=torch.int32, device=dev)
    need = native.mg_gemm_i8_workspace_size(n, n, n)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    q = native.mg_i8_packed_size(n, n)
    qA, qB = ws[:q], ws[need - q:]
    fp16 = bench.gemm_call("fp16", "N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)

    def i8_full():
        native.check(native.mg_gemm_i8("N", "N", n, n, n, 1, Ai.data_ptr(), n, Bi.data_ptr(), n, 0, Ci.data_ptr(),
                                       n, ws.data_ptr(), need, sp), "mg_gemm_i8")

    def i8_gemm():
        native.check(native.mg_gemm_i8_packed(n, n, n, 1, qA.data_ptr(), qB.data_ptr(), 0, Ci.data_ptr(), n, sp),
                     "mg_gemm_i8_packed")

    i8_full()
    cases = {"fp16": fp16, "int8_end_to_end": i8_full, "int8_gemm_only": i8_gemm}
    per = {c: [] for c in cases}
    clk = {c: [] for c in cases}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for c in bench.shuffled(cases):
            r = bench.case(cases[c])
            per[c] += r["per_ms"]
            clk[c].append([r["sclk_mhz_during"], r["sclk_mhz"]])
    I, J = si.sample_indices(n, n, 512, 306)
    Cf = torch.zeros(n * n, device=dev)
    bench.gemm_call("fp16", "N", "N", n, n, n, 1.0, A, n, B, n, 0.0, Cf, n, ws=fp16.workspace)()
    got16 = bench.gather(Cf, n, I, J)
    Ci.zero_()
    i8_full()
    got8 = Ci.reshape(-1)[torch.from_numpy(I * n + J).to(dev)].cpu().numpy()
    mism = oracle_i8_mismatches(a8, b8, 1, got8, I, J)
    ms = {c: float(np.mean(per[c])) for c in cases}

    def i8_row(c, cfg=None):
        r = {"ms": round(ms[c], 4), "tops": round(tflops(flops, ms[c]), 1),
             "frac_of_int8_peak": round(tflops(flops, ms[c]) / INT8_PEAK_TOPS, 3), "step_ms": stats(per[c]),
             "sclk_mhz": clk[c], "sampled_mismatches_vs_integer_oracle": mism, "samples": len(I)}
        if cfg is not None:
            r["config"] = cfg
        return r

    rows = {
        "fp16": {"ms": round(ms["fp16"], 4), "tflops": round(tflops(flops, ms["fp16"]), 1),
                 "frac_of_fp16_peak": round(tflops(flops, ms["fp16"]) / PEAK_TFLOPS["bf16"], 3),
                 "config": native.mg_tuned_config(4, n, n, n), "step_ms": stats(per["fp16"]), "sclk_mhz": clk["fp16"],
                 "sampled_error_vs_fp64_oracle": oracle_error("N", "N", n, n, n, 1.0, a16, n, b16, n, 0.0, None,
                                                              got16, I, J), "tolerance": TOL["fp16"]},
        "int8_end_to_end": i8_row("int8_end_to_end"),
        "int8_gemm_only": i8_row("int8_gemm_only", native.mg_tuned_config(5, n, n, n)),
    }
    g = rows["int8_gemm_only"]
    out = header(bench, "FP16 TFLOP/s and INT8 TOP/s at 8192^3", "TOP/s", g["tops"], g["ms"], "i8",
                 {"workload": "fp16_int8_8192x8192x8192_nn", "fp16_inputs": "uniform[-1,1] float32",
                  "int8_inputs": "uniform integers in [-128, 127]", "rounds": args.rounds})
    out["roofline"] = {"bound": "mfma", "achieved": g["tops"], "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                       "frac": g["frac_of_int8_peak"], "traffic": None,
                       "kernel": tuned_kernel_name(native, 5, "gemm_i8_direct_kernel", n, n, n)}
    out["rows"] = rows
    return out


def bench_smallk(bench, si):
    """The small-K shape of the FP32 sweep, 8192 x 8192 x 256 NN (alpha 1.5,
    beta 0.5, U[-1, 1]), on the FP32 and bf16x3 paths.  Algorithmic HBM bytes
    per launch: 4(MK + KN) + 8MN (A and B read once, C0 read, C written).
    Timed warm (back-to-back launches, operands partly left in the 256 MB
    Infinity Cache by the previous launch) and flushed (a 512 MB buffer
    written between launches, each launch between its own events)."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    m, n, k = SMALLK_SHAPE
    a = si.uniform((m * k,), si.seed_for(2, "A"))
    b = si.uniform((k * n,), si.seed_for(2, "B"))
    c0 = si.uniform((m * n,), si.seed_for(2, "C"))
    A, B, C0 = (torch.from_numpy(x).to(dev) for x in (a, b, c0))
    flush_buf = torch.empty(512 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    flops = 2.0 * m * n * k
    nbytes = 4.0 * (m * k + k * n) + 8.0 * m * n
    C = C0.clone()
    runs = {p: bench.gemm_call(p, "N", "N", m, n, k, ALPHA, A, k, B, n, BETA, C, n) for p in ("fp32", "bf16x3")}
    cases = [(p, mode) for p in runs for mode in ("warm", "flushed")]
    per = {c: [] for c in cases}
    clk = {c: [] for c in cases}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for case in bench.shuffled(cases):
            p, mode = case
            run = runs[p]
            bench.warm(run, args.warmup)
            if mode == "warm":
                t, _, _ = bench.steps(run, args.steps)
            else:
                t = bench.per_launch(run, args.steps, between=lambda: flush_buf.fill_(1.0))
            per[case] += t
            clk[case].append(bench.sclk())
    I, J = si.sample_indices(m, n, SAMPLES, 307)
    rows = {}
    for p in runs:
        Cf = C0.clone()
        bench.gemm_call(p, "N", "N", m, n, k, ALPHA, A, k, B, n, BETA, Cf, n, ws=runs[p].workspace)()
        got = bench.gather(Cf, n, I, J)
        err = oracle_error("N", "N", m, n, k, ALPHA, a, k, b, n, BETA, c0, got, I, J)
        st, cfg, splits, packed = native.mg_gemm_plan(PATH_ID[p], m, n, k, runs[p].workspace.numel())
        rows[p] = {"config": cfg, "splits": splits, "prepacked": packed, "sampled_error_vs_fp64_oracle": err}
        for mode in ("warm", "flushed"):
            ms = float(np.median(per[(p, mode)]))
            rows[p][mode] = {"ms": round(ms, 5), "tflops": round(tflops(flops, ms), 2),
                             "algorithmic_gbps": round(nbytes / ms / 1e6, 1),
                             "frac_of_hbm_peak": round(nbytes / ms / 1e6 / 8000.0, 3),
                             "step_ms": stats(per[(p, mode)]), "sclk_mhz": clk[(p, mode)]}
    f = rows["fp32"]["warm"]
    traffic = measured_traffic(PROFILE_SMALLK)
    out = header(bench, "FP32 SGEMM TFLOP/s and HBM GB/s at 8192x8192x256", "TFLOP/s", f["tflops"], f["ms"], "f32",
                 {"workload": "sgemm_small_k_8192x8192x256_nn", "M": m, "N": n, "K": k, "layout": "NN",
                  "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]", "rounds": args.rounds})
    out["roofline"] = {"bound": "mfma", "achieved": f["tflops"], "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                       "frac": round(f["tflops"] / PEAK_TFLOPS["fp32"], 4), "traffic": traffic,
                       "kernel": "the FP32 kernel of the plan in rows.fp32.config",
                       "algorithmic_bytes_per_launch": nbytes,
                       "hbm_gbps_measured": None if traffic is None else round(traffic / f["ms"] / 1e6, 1)}
    out["rows"] = rows
    return out


def bench_syr2k(bench, si):
    """SYR2K (Section 5.1) on the lower triangle, N = K = 8192, trans 'N',
    alpha 1.5, beta 0.5: one launch over the triangle's tiles, both products
    in one accumulator.  Work counted as 2*N^2*K (the triangle's N(N+1)/2
    entries, two K-long dot products each).  Beside it, the same update done
    with two full FP32 GEMMs (C += alpha*A*B^T, then C += alpha*B*A^T over the
    whole square), the way it would be written without SYR2K."""
    torch, native, dev, args = bench.torch, bench.native, bench.dev, bench.args
    sp = bench.sp
    n = k = M
    x = si.uniform((n * k,), si.seed_for(5, "X"))
    y = si.uniform((n * k,), si.seed_for(5, "W1"))
    c0 = si.uniform((n * n,), si.seed_for(5, "C"))
    X, Y, C0 = (torch.from_numpy(v).to(dev) for v in (x, y, c0))
    C = C0.clone()
    need = native.mg_syr2k_workspace_size(0, n, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

    def syr2k_fn(splits, Cd):
        def run():
            native.check(native.mg_force_splits(0, splits), "mg_force_splits")
            try:
                w = native.mg_syr2k_workspace_size(0, n, k)
                native.check(native.mg_syr2k(0, "L", "N", n, k, ALPHA, X.data_ptr(), k, Y.data_ptr(), k, BETA,
                                             Cd.data_ptr(), n, ws.data_ptr(), w, sp), "mg_syr2k")
            finally:
                native.mg_force_splits(0, -1)
        return run

    def two_gemms():
        native.check(native.mg_gemm(0, "N", "T", n, n, k, ALPHA, X.data_ptr(), k, Y.data_ptr(), k, BETA,
                                    C.data_ptr(), n, None, 0, sp), "mg_gemm")
        native.check(native.mg_gemm(0, "N", "T", n, n, k, ALPHA, Y.data_ptr(), k, X.data_ptr(), k, 1.0,
                                    C.data_ptr(), n, None, 0, sp), "mg_gemm")

    cases = {"syr2k": syr2k_fn(-1, C), "syr2k_unsplit": syr2k_fn(1, C), "two_full_gemms": two_gemms}
    per = {c: [] for c in cases}
    clk = {c: [] for c in cases}
    for rnd in range(args.rounds):
        progress(f"round {rnd + 1}/{args.rounds}")
        for c in bench.shuffled(cases):
            r = bench.case(cases[c], steps=args.steps if c != "two_full_gemms" else max(2, args.steps // 2))
            per[c] += r["per_ms"]
            clk[c].append([r["sclk_mhz_during"], r["sclk_mhz"]])
    Cf = C0.clone()
    syr2k_fn(-1, Cf)()
    I, J = si.sample_indices(n, n, 2 * SAMPLES, 308)
    low = I >= J
    I, J = I[low], J[low]
    got = bench.gather(Cf, n, I, J)
    upper_untouched = bool(torch.equal(torch.triu(Cf.view(n, n), 1), torch.triu(C0.view(n, n), 1)))
    err = oracle_syr2k_error("N", k, ALPHA, x, y, k, BETA, c0, n, got, I, J)
    flops = 2.0 * n * n * k
    ms = float(np.mean(per["syr2k"]))
    tf = tflops(flops, ms)
    st, plan_cfg, auto_splits = native.mg_syr2k_plan(0, n, k)
    native.check(st, "mg_syr2k_plan")
    info = native.mg_config_info(0, plan_cfg)
    out = header(bench, "SYR2K TFLOP/s (2*N^2*K useful flops) at N = K = 8192", "TFLOP/s", round(tf, 2),
                 round(ms, 4), "f32", {"workload": "ssyr2k_lower_n_8192x8192", "N": n, "K": k, "uplo": "L",
                                       "trans": "N", "alpha": ALPHA, "beta": BETA, "inputs": "uniform[-1,1]",
                                       "rounds": args.rounds})
    out["roofline"] = {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                       "frac": round(tf / PEAK_TFLOPS["fp32"], 4), "traffic": None,
                       "kernel": f"syr2k_kernel<{info['bm']},{info['bk']},{info['wm']},{info['wn']}> "
                                 f"(configuration {plan_cfg}, split {auto_splits})"}
    out["step_ms"] = {c: stats(v) for c, v in per.items()}
    out["sclk_mhz"] = clk
    out["splits"] = int(auto_splits)
    out["unsplit_ms"] = round(float(np.mean(per["syr2k_unsplit"])), 4)
    ms2 = float(np.mean(per["two_full_gemms"]))
    out["two_full_gemms"] = {"ms": round(ms2, 4), "speedup_of_syr2k": round(ms2 / ms, 3)}
    out["sampled_error_vs_fp64_oracle"] = err
    out["upper_triangle_untouched"] = upper_untouched
    return out


if __name__ == "__main__":
    main()
