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

Usage (on a GPU):
    python -m paper_2305_18236_amd.autotune --mode batched --paths fp32,bf16x3,bf16 \
        --out paper_2305_18236_amd/tuning_table.txt
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

from . import _native

PATH_IDS = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["batched", "single"], default="batched")
    ap.add_argument("--paths", default="fp32,bf16x3,bf16")
    ap.add_argument("--min-bucket", type=int, default=5)
    ap.add_argument("--max-bucket", type=int, default=11)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    os.environ["MGEMM_TUNING"] = "none"   # measure the candidates, not a previous table
    tune(tuple(a.paths.split(",")), a.mode, range(a.min_bucket, a.max_bucket + 1), a.reps, a.out)


if __name__ == "__main__":
    main()
