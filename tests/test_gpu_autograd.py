"""Differentiation through the library: GemmFn's hand-written backward
(dA = dC B^T, dB = A^T dC on the transposed-operand kernels) checked against
central finite differences of the GPU forward and against the FP64 oracle's
gradients of loss = sum(Y * G), Y = (X W1) W2.
"""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu


def _chain_inputs(Mx, D, Hd, seed_cfg=5):
    X = si.uniform((Mx, D), si.seed_for(seed_cfg, "X"))
    W1 = si.uniform((D, Hd), si.seed_for(seed_cfg, "W1"))
    W2 = si.uniform((Hd, D), si.seed_for(seed_cfg, "W2"))
    G = si.gaussian((Mx, D), si.seed_for(seed_cfg, "G"))
    return X, W1, W2, G


def _gpu_grads(X, W1, W2, G, dev, path):
    from paper_2305_18236_amd.autograd import chain
    tX, tW1, tW2 = (torch.from_numpy(a).to(dev).requires_grad_(True) for a in (X, W1, W2))
    tG = torch.from_numpy(G).to(dev)
    Y = chain(tX, tW1, tW2, path)
    Y.backward(tG)    # d(sum(Y * G))/dY = G
    torch.cuda.synchronize()
    return Y.detach().cpu().numpy(), {k: t.grad.cpu().numpy().astype(np.float64)
                                      for k, t in (("dX", tX), ("dW1", tW1), ("dW2", tW2))}


@pytest.mark.parametrize("path", ["bf16x3", "fp32"])
def test_small_chain_against_oracle_and_finite_differences(gpu, path):
    """The 64 x 32 x 32 instance: X 64x32, W1 32x32, W2 32x32, G 64x32."""
    from paper_2305_18236_amd.autograd import chain
    X, W1, W2, G = _chain_inputs(64, 32, 32)
    _, g = _gpu_grads(X, W1, W2, G, gpu, path)
    ref, den = oracle.chain_grads(X, W1, W2, G)
    for k in ref:
        err = oracle.normalized_error(g[k], ref[k], den[k])
        assert err <= 1e-4, (path, k, err)   # two stacked GEMMs at K = 32 (worst case 2 x 5e-5)

    # Central differences of the GPU forward, eps = 1e-3.  The loss is linear in
    # every single entry, so the difference quotient has no truncation error:
    # what is left is the forward's rounding, divided by 2*eps.
    tX, tW1, tW2 = (torch.from_numpy(a).to(gpu) for a in (X, W1, W2))
    Gd = G.astype(np.float64)
    eps = 1e-3

    def loss(a, b, c):
        with torch.no_grad():
            Y = chain(a, b, c, path)
        return float(np.sum(Y.cpu().numpy().astype(np.float64) * Gd))

    rng = np.random.default_rng(0)
    for name, t, idx_shape in (("dX", tX, X.shape), ("dW1", tW1, W1.shape), ("dW2", tW2, W2.shape)):
        flat = rng.choice(int(np.prod(idx_shape)), size=96, replace=False)
        worst = 0.0
        for f in flat:
            i, j = divmod(int(f), idx_shape[1])
            orig = t[i, j].item()
            t[i, j] = orig + eps
            xp = t[i, j].item()          # the perturbed values as stored (float32)
            lp = loss(tX, tW1, tW2)
            t[i, j] = orig - eps
            xm = t[i, j].item()
            lm = loss(tX, tW1, tW2)
            t[i, j] = orig
            fd = (lp - lm) / (xp - xm)
            worst = max(worst, abs(fd - g[name][i, j]))
        scale = np.max(np.abs(g[name]))
        assert worst <= 1e-2 * scale, (path, name, worst, scale)


def test_backward_reads_transposed_layouts_without_copies(gpu):
    """GemmFn's backward on stored layouts equals explicit GEMMs on contiguous
    transposed copies, bit for bit (packing makes every layout look the same
    to the micro-kernel)."""
    from paper_2305_18236_amd import gemm
    from paper_2305_18236_amd.autograd import GemmFn
    A = torch.from_numpy(si.uniform((300, 200), 1)).to(gpu).requires_grad_(True)
    B = torch.from_numpy(si.uniform((200, 260), 2)).to(gpu).requires_grad_(True)
    dC = torch.from_numpy(si.gaussian((300, 260), 3)).to(gpu)
    C = GemmFn.apply(A, B, "fp32")
    C.backward(dC)
    dA_ref = gemm(dC, B.detach().t().contiguous())
    dB_ref = gemm(A.detach().t().contiguous(), dC)
    torch.cuda.synchronize()
    assert torch.equal(A.grad, dA_ref) and torch.equal(B.grad, dB_ref)


@pytest.mark.slow
def test_full_size_chain_sampled(gpu):
    """X 4096x2048, W1 2048x8192, W2 8192x2048, bf16x3 forward and backward;
    sampled FP64 oracle values of Y and every gradient, normalised by the
    chained denominators (two stacked GEMMs: 2 x 1e-5)."""
    X, W1, W2, G = _chain_inputs(4096, 2048, 8192)
    Y, g = _gpu_grads(X, W1, W2, G, gpu, "bf16x3")
    samples = oracle.chain_entries(X, W1, W2, G)
    for name, (I, J, ref, den) in samples.items():
        got = Y[np.ix_(I, J)].astype(np.float64) if name == "Y" else g[name][np.ix_(I, J)]
        err = oracle.normalized_error(got, ref, den)
        print(f"chain {name}: sampled normalised error {err:.3e}")
        assert err <= 2e-5, (name, err)
