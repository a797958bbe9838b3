"""Autotuner: choose the tile configuration per shape bucket by measurement.

The paper fixes the cache-blocking parameters mc/kc/nc from a cache model
(Section 3.1, Eq. 1-7) and leaves only the register tile mr/nr/kr to tuning.
On the GPU every level is a tile-shape choice (workgroup tile BM x BN, panel
depth BK, wave tile WM x WN), so all of them are chosen here, per shape bucket,
by timing the candidates that survive an analytic pruning step (the Eq. 1-7
analogue: LDS capacity and register budget are fixed per configuration at
build time; a candidate is dropped when its tiles would pad the problem to more
than 4x its area, i.e. waste three quarters of the matrix-core work).

Buckets are round(log2) of M, N and K, the same rule the C library uses to
read the table.  Two modes:
  batched: candidates are the tile variants of the persistent batched kernel;
           each is timed inside the persistent kernel on a batch of copies of
           the bucket's representative shape, with enough copies for about
           four 128 x 128 tiles per workgroup slot of the GPU, i.e. in the
           saturated regime a large uneven batch runs in (a lone problem
           would favour small tiles just to occupy more compute units);
  single:  candidates are all configurations of the path, timed on one GEMM.

  exact:   for each given shape (default: the benchmark workloads' shapes),
           the candidates the blocking model admits (blocking.py, the
           Eq. 1-7 analogue: LDS, register file, L2 / Infinity Cache,
           divisibility, rounds over the compute units) plus the library's
           current plan, each a (configuration, K ranges) pair, timed on one
           GEMM; the fastest becomes an exact-shape line "path M N K config x
           splits", which single GEMMs of that shape read before any bucket.

Usage (on a GPU):
    python -m paper_2305_18236_amd.autotune --mode batched --paths fp32,bf16x3,bf16 \
        --out paper_2305_18236_amd/tuning_table.txt
    python -m paper_2305_18236_amd.autotune --mode exact --paths fp32,bf16x3,bf16,fp16,fp8,int8 \
        --merge paper_2305_18236_amd/tuning_table.txt
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

from . import _native, blocking

PATH_IDS = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4, "int8": 5}
# A measured plan replaces the rule's only when it is this much faster
# (repeated runs of one plan differ by 1-2 %).
NOISE = 1.03

# The benchmark workloads' shapes: the small case, the FP32 sweep, the shapes
# whose workgroups do not fall into whole rounds, and the six products of the
# differentiable chain (X 4096x2048, W1 2048x8192, W2 8192x2048).
EXACT_SHAPES = [(256, 256, 256), (1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096),
                (8192, 8192, 8192), (8192, 8192, 256), (256, 8192, 8192), (16384, 1024, 4096),
                (1536, 1536, 1536), (3072, 3072, 3072), (6144, 6144, 6144), (3072, 3072, 1024),
                (4096, 8192, 2048), (4096, 2048, 8192), (8192, 2048, 4096), (2048, 8192, 4096)]
SLOTS = 512          # workgroup slots of the persistent kernel: 256 CUs x 2
BATCHED_CFGS = {0: [3, 0], 1: [4, 5, 2], 2: [4, 5, 2], 4: [4, 5, 2]}


def bucket(x: int) -> int:
    """round(log2 x) with the C library's tie rule (x >= 1.5 * 2^b rounds up)."""
    if x <= 1:
        return 0
    b = x.bit_length() - 1
    if 2 * x >= 3 << b:
        b += 1
    return min(b, 20)


def padded_area_ratio(M, N, bm, bn) -> float:
    return (math.ceil(M / bm) * bm * math.ceil(N / bn) * bn) / float(M * N)


def candidates(path_id: int, mode: str, M: int, N: int):
    ids = BATCHED_CFGS[path_id] if mode == "batched" else list(range(_native.mg_num_configs(path_id)))
    out = []
    for cid in ids:
        c = _native.mg_config_info(path_id, cid)
        if padded_area_ratio(M, N, c["bm"], c["bn"]) <= 4.0:
            out.append(cid)
    if not out:   # keep the smallest tile
        out = [min(ids, key=lambda i: _native.mg_config_info(path_id, i)["bm"] * _native.mg_config_info(path_id, i)["bn"])]
    return out


class _Bench:
    def __init__(self, torch, dev):
        self.torch = torch
        self.dev = dev

    def operands(self, M, N, K, copies):
        """`copies` problems sharing one A and one B, each with its own slice of C."""
        t = self.torch
        g = t.Generator(device=self.dev)
        g.manual_seed(M * 7919 + N * 31 + K)
        A = t.rand((M, K), device=self.dev, generator=g) * 2 - 1
        B = t.rand((K, N), device=self.dev, generator=g) * 2 - 1
        C = t.zeros((copies, M, N), device=self.dev)
        return [(A, B, C[i]) for i in range(copies)]

    def time(self, fn, reps):
        t = self.torch
        fn()
        t.cuda.synchronize()
        e0 = t.cuda.Event(enable_timing=True)
        e1 = t.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            t.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best


def tune(paths=("fp32", "bf16x3", "bf16"), mode="batched", buckets=range(5, 12), reps=3, out=None,
         log=sys.stdout):
    import torch
    from . import gemm, gemm_batched
    dev = torch.device("cuda:0")
    _native.lib()
    bench = _Bench(torch, dev)
    lines = ["# mgemm tuning table: path mb nb kb config mode (mb/nb/kb = round(log2 M/N/K);",
             "# mode b: read by the batched kernel, s: by single GEMMs)",
             f"# mode {mode}, written by paper_2305_18236_amd.autotune on {time.strftime('%Y-%m-%d')}"]
    t0 = time.time()
    for path in paths:
        pid = PATH_IDS[path]
        for mb in buckets:
            for nb in buckets:
                for kb in buckets:
                    M, N, K = 2 ** mb, 2 ** nb, 2 ** kb
                    tiles128 = math.ceil(M / 128) * math.ceil(N / 128)
                    copies = 1 if mode == "single" else int(min(4096, max(1, math.ceil(4 * SLOTS / tiles128))))
                    ops = bench.operands(M, N, K, copies)
                    best, best_t = None, float("inf")
                    for cid in candidates(pid, mode, M, N):
                        assert _native.mg_force_config(pid, cid) == 0
                        try:
                            if mode == "batched":
                                probs = [(A, B, C, 1.0, 0.0) for A, B, C in ops]
                                ms = bench.time(lambda: gemm_batched(probs, path=path), reps)
                            else:
                                A, B, C = ops[0]
                                ms = bench.time(lambda: gemm(A, B, C, path=path), reps)
                        finally:
                            _native.mg_force_config(pid, -1)
                        if ms < best_t:
                            best, best_t = cid, ms
                    lines.append(f"{pid} {mb} {nb} {kb} {best} {'b' if mode == 'batched' else 's'}")
                    tflops = 2.0 * M * N * K * copies / (best_t * 1e-3) / 1e12
                    print(f"{path} M{M} N{N} K{K} x{copies}: config {best} {best_t * 1e3:.1f} us "
                          f"{tflops:.1f} TFLOP/s", file=log, flush=True)
    print(f"tuned in {time.time() - t0:.1f} s", file=log, flush=True)
    text = "\n".join(lines) + "\n"
    if out:
        with open(out, "w") as f:
            f.write(text)
    return text


def _plan_now(pid, M, N, K):
    """(config, K ranges) the library runs now for this shape with a full workspace."""
    if pid == 5:
        return _native.mg_tuned_config(5, M, N, K), 1
    need = _native.mg_gemm_workspace_size(pid, "N", "N", M, N, K)
    st, cfg, splits, _ = _native.mg_gemm_plan(pid, M, N, K, need)
    return cfg, splits


def tune_exact(paths, shapes=EXACT_SHAPES, reps=5, log=sys.stdout):
    """Exact-shape lines for `shapes` on `paths` (see the module docstring)."""
    import torch
    dev = torch.device("cuda:0")
    _native.lib()
    stream = torch.cuda.current_stream().cuda_stream
    lines = []
    for path in paths:
        pid = PATH_IDS[path]
        cfgs = blocking.library_configs(_native, pid)
        for (M, N, K) in shapes:
            if pid == 5:
                A = torch.randint(-128, 128, (M * K,), dtype=torch.int8, device=dev)
                B = torch.randint(-128, 128, (K * N,), dtype=torch.int8, device=dev)
                C = torch.zeros(M * N, dtype=torch.int32, device=dev)
            else:
                A = torch.rand(M * K, device=dev) * 2 - 1
                B = torch.rand(K * N, device=dev) * 2 - 1
                C = torch.rand(M * N, device=dev) * 2 - 1
            default = _plan_now(pid, M, N, K)
            cands = blocking.candidates(cfgs, M, N, K, keep=32)
            if default not in cands:
                cands.append(default)
            results = []
            for cfg, splits in cands:
                assert _native.mg_force_config(pid, cfg) == 0
                if pid != 5:   # INT8 has no split
                    assert _native.mg_force_splits(pid, splits) == 0
                try:
                    if pid == 5:
                        need = _native.mg_gemm_i8_workspace_size(M, N, K)
                    else:
                        need = _native.mg_gemm_workspace_size(pid, "N", "N", M, N, K)
                    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

                    if pid == 5:
                        def run():
                            _native.check(_native.mg_gemm_i8("N", "N", M, N, K, 1, A.data_ptr(), K, B.data_ptr(), N,
                                                             0, C.data_ptr(), N, ws.data_ptr(), need, stream),
                                          "mg_gemm_i8")
                    else:
                        def run():
                            _native.check(_native.mg_gemm(pid, "N", "N", M, N, K, 1.5, A.data_ptr(), K, B.data_ptr(),
                                                          N, 0.5, C.data_ptr(), N, ws.data_ptr(), need, stream),
                                          "mg_gemm")
                    ms = _time_launches(torch, run, reps)
                finally:
                    _native.mg_force_config(pid, -1)
                    if pid != 5:
                        _native.mg_force_splits(pid, -1)
                results.append((ms, cfg, splits))
            results.sort()
            ms, cfg, splits = results[0]
            dms = [r[0] for r in results if (r[1], r[2]) == default][0]
            if dms < NOISE * ms:
                # within run-to-run noise of the rule's plan: keep the rule's
                ms, cfg, splits = dms, default[0], default[1]
            lines.append(f"{pid} {M} {N} {K} {cfg} x {splits}")
            print(f"{path} {M}x{N}x{K}: config {cfg} splits {splits} {ms * 1e3:.1f} us "
                  f"({2.0 * M * N * K / ms / 1e9:.1f} TFLOP/s); rule's plan {default} {dms * 1e3:.1f} us; "
                  f"{len(results)} candidates", file=log, flush=True)
            del A, B, C
    return lines


def _time_launches(torch, run, reps):
    """Median time of one launch: warm up for about 30 ms, then `reps` blocks
    of launches between HIP events (enough launches per block for ~2 ms)."""
    t0 = time.perf_counter()
    n = 0
    while n < 3 or (time.perf_counter() - t0) < 0.03:
        run()
        n += 1
        if n % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run()
    e1.record()
    torch.cuda.synchronize()
    per = max(e0.elapsed_time(e1), 1e-3)
    count = max(1, min(50, int(2.0 / per)))
    out = []
    for _ in range(reps):
        e0.record()
        for _ in range(count):
            run()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / count)
    out.sort()
    return out[len(out) // 2]


def merge_exact(table_path, new_lines):
    """Replace the exact-shape lines of `table_path` for the shapes in
    new_lines (same path, M, N, K); keep every other line."""
    keys = {tuple(l.split()[:4]) for l in new_lines}
    kept = []
    if os.path.exists(table_path):
        for line in open(table_path):
            f = line.split()
            if len(f) >= 6 and not line.lstrip().startswith("#") and f[5] == "x" and tuple(f[:4]) in keys:
                continue
            kept.append(line.rstrip("\n"))
    stamp = f"# exact-shape lines (mode x: path M N K config x splits), measured {time.strftime('%Y-%m-%d')}"
    kept = [l for l in kept if not l.startswith("# exact-shape lines")]
    with open(table_path, "w") as f:
        f.write("\n".join(kept + [stamp] + list(new_lines)) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["batched", "single", "exact"], default="batched")
    ap.add_argument("--paths", default="fp32,bf16x3,bf16")
    ap.add_argument("--min-bucket", type=int, default=5)
    ap.add_argument("--max-bucket", type=int, default=11)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--merge", default=None, help="exact mode: table file whose exact lines are replaced")
    a = ap.parse_args(argv)
    os.environ["MGEMM_TUNING"] = "none"   # measure the candidates, not a previous table
    if a.mode == "exact":
        lines = tune_exact(tuple(a.paths.split(",")), reps=max(a.reps, 5))
        if a.merge:
            merge_exact(a.merge, lines)
        if a.out:
            with open(a.out, "w") as f:
                f.write("\n".join(lines) + "\n")
        return
    tune(tuple(a.paths.split(",")), a.mode, range(a.min_bucket, a.max_bucket + 1), a.reps, a.out)


if __name__ == "__main__":
    main()
