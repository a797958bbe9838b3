"""GPU parity of the uneven batched GEMM (one persistent launch) against the
FP64 oracle, per problem, and bitwise against one launch per problem with the
same tile configuration."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from helpers import Problem, tolerance

pytestmark = pytest.mark.gpu

PATHS = ["fp32", "bf16x3", "bf16"]
PID = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp16": 4}


def _run_batched(probs, path, dev):
    from paper_2305_18236_amd import _native
    arr = (_native.mg_problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = _native.mg_problem(p.tA.encode(), p.tB.encode(), p.M, p.N, p.K, p.alpha, p.beta,
                                    p.dA.data_ptr(), p.lda, p.dB.data_ptr(), p.ldb, p.dC.data_ptr(), p.ldc)
    need = _native.mg_gemm_batched_workspace_size(PID[path], len(probs))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st, bad = _native.mg_gemm_batched(PID[path], len(probs), arr, ws.data_ptr(), need,
                                      torch.cuda.current_stream().cuda_stream)
    assert st == 0, (_native.status_string(st), bad)


def _mixed_batch(seed, count=40):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        M, N, K = (int(x) for x in rng.integers(1, 300, 3))
        tA, tB = rng.choice(["N", "T"]), rng.choice(["N", "T"])
        alpha, beta = float(rng.choice([1.0, 1.5, -0.5])), float(rng.choice([0.0, 0.5, 1.0]))
        probs.append(Problem(M, N, K, tA, tB, alpha, beta, seed=seed * 100 + i))
    # edge cases inside one batch: empty, K = 0, alpha = 0, a 1x1x1 and a multi-tile problem
    probs.append(Problem(0, 7, 5, seed=seed * 100 + 90))
    probs.append(Problem(9, 0, 5, seed=seed * 100 + 91))
    probs.append(Problem(17, 19, 0, alpha=1.0, beta=0.5, seed=seed * 100 + 92))
    probs.append(Problem(33, 35, 37, alpha=0.0, beta=0.5, seed=seed * 100 + 93))
    probs.append(Problem(1, 1, 1, seed=seed * 100 + 94))
    probs.append(Problem(700, 650, 500, "T", "N", 1.0, 0.5, seed=seed * 100 + 95))
    return probs


@pytest.mark.parametrize("path", PATHS)
def test_mixed_batch_parity(gpu, path):
    probs = [p.to_device(gpu) for p in _mixed_batch(7)]
    _run_batched(probs, path, gpu)
    for p in probs:
        if p.M == 0 or p.N == 0:
            assert p.padding_untouched()
            continue
        C = p.result()
        Cref, D = p.oracle()
        err = oracle.normalized_error(C, Cref, D)
        assert err <= tolerance(path, p.K), (path, p.M, p.N, p.K, p.tA, p.tB, err)
        assert p.padding_untouched()


@pytest.mark.parametrize("path", PATHS)
def test_batched_equals_single_launches_bitwise(gpu, path):
    """Each problem in the batch runs the same tile code as a single launch
    with its configuration, so the results are identical bit for bit."""
    from paper_2305_18236_amd import _native
    probs = [p.to_device(gpu) for p in _mixed_batch(11, count=24)]
    _run_batched(probs, path, gpu)
    batched = [p.result() for p in probs]
    for p, Cb in zip(probs, batched):
        if p.M == 0 or p.N == 0:
            continue
        p.reset_c()
        cfg = _native.mg_batched_config(PID[path], p.M, p.N, p.K)
        assert _native.mg_force_config(PID[path], cfg) == 0
        try:
            assert p.run(path) == 0
        finally:
            _native.mg_force_config(PID[path], -1)
        assert np.array_equal(p.result(), Cb), (path, p.M, p.N, p.K, cfg)


@pytest.mark.parametrize("path", ["fp32", "bf16x3"])
def test_uneven_512_workload_sampled(gpu, path):
    """The uneven workload: 512 problems, M, N, K log-uniform in [32, 2048]
    (multiples of 8), U[-1, 1]; 64 sampled outputs per problem against the oracle."""
    sizes = si.batched_sizes(512, si.seed_for(4, "A"))
    probs = []
    for i, (M, N, K) in enumerate(sizes):
        p = Problem.from_arrays(si.uniform((M, K), si.seed_for(4, "A", i)),
                                si.uniform((K, N), si.seed_for(4, "B", i)))
        probs.append(p.to_device(gpu))
    _run_batched(probs, path, gpu)
    worst = 0.0
    for i, p in enumerate(probs):
        C = p.result()
        I, J = si.sample_indices(p.M, p.N, 64, i)
        cref, d = p.oracle_entries(I, J)
        worst = max(worst, oracle.normalized_error(C[I, J], cref, d))
    print(f"{path}: worst sampled normalised error over 512 problems {worst:.3e}")
    assert worst <= tolerance(path, 32)


@pytest.mark.parametrize("path", ["fp32", "bf16x3"])
def test_timed_launch_matches_and_stamps_are_valid(gpu, path):
    """mg_gemm_batched_timed computes what mg_gemm_batched computes (bit for
    bit) and records a start and end wall-clock stamp per workgroup."""
    from paper_2305_18236_amd import _native
    pid = PID[path]
    probs = [p.to_device(gpu) for p in _mixed_batch(13, count=30)]
    _run_batched(probs, path, gpu)
    plain = [p.result() for p in probs]
    for p in probs:
        p.reset_c()
    arr = (_native.mg_problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = _native.mg_problem(p.tA.encode(), p.tB.encode(), p.M, p.N, p.K, p.alpha, p.beta,
                                    p.dA.data_ptr(), p.lda, p.dB.data_ptr(), p.ldb, p.dC.data_ptr(), p.ldc)
    need = _native.mg_gemm_batched_workspace_size(pid, len(probs))
    ws = torch.empty(need, dtype=torch.uint8, device=gpu)
    slots = _native.mg_batched_slots(pid)
    assert slots >= 256
    stamps = torch.zeros(2 * slots, dtype=torch.int64, device=gpu)
    sp = torch.cuda.current_stream().cuda_stream
    # stamps missing or too short: rejected on the host, nothing launched
    assert _native.mg_gemm_batched_timed(pid, len(probs), arr, ws.data_ptr(), need, sp, None, 2 * slots)[0] == -8
    assert _native.mg_gemm_batched_timed(pid, len(probs), arr, ws.data_ptr(), need, sp, stamps.data_ptr(),
                                         2 * slots - 1)[0] == -8
    st, bad, grid = _native.mg_gemm_batched_timed(pid, len(probs), arr, ws.data_ptr(), need, sp,
                                                  stamps.data_ptr(), 2 * slots)
    assert st == 0, (_native.status_string(st), bad)
    for p, Cp in zip(probs, plain):
        if p.M and p.N:
            assert np.array_equal(p.result(), Cp), (path, p.M, p.N, p.K)
    t = stamps.cpu().numpy().reshape(-1, 2)
    assert 0 < grid <= slots
    start, end = t[:grid, 0], t[:grid, 1]
    assert (start > 0).all() and (end >= start).all()
    assert (t[grid:] == 0).all()              # workgroups beyond the grid do not exist
    hz = _native.mg_wall_clock_hz()
    assert hz > 0
    span = (end.max() - start.min()) / hz
    assert 0 < span < 1.0, span              # a few microseconds to milliseconds


def test_timed_launch_of_empty_batch(gpu):
    from paper_2305_18236_amd import _native
    slots = _native.mg_batched_slots(0)
    stamps = torch.zeros(2 * slots, dtype=torch.int64, device=gpu)
    arr = (_native.mg_problem * 1)()
    st, bad, grid = _native.mg_gemm_batched_timed(0, 0, arr, None, 0, torch.cuda.current_stream().cuda_stream,
                                                  stamps.data_ptr(), 2 * slots)
    assert (st, grid) == (0, 0)
    assert int(stamps.abs().sum()) == 0
