"""GPU warm-start MLP (BF16 operands on MFMA, FP32 accumulation) vs the FP64
numpy oracle.  Tolerances follow from BF16 rounding (8 significand bits,
relative 2^-8 per operand): outputs within 3e-2 of the output scale, gradient
direction cosine >= 0.999 per layer."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    return torch


def _mlp(sizes, batch, seed=0):
    from paper_2311_07710_amd.mlp import MLP, init_params
    m = MLP(sizes, max_batch=batch)
    p = init_params(sizes, seed=seed, out_scale=1.0)
    m.set_params(p)
    return m, p


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


@pytest.mark.parametrize("sizes,batch", [([37, 64, 48, 29], 50), ([8, 5], 3), ([100, 130, 70], 129)])
def test_forward_backward_match_oracle(torch_cuda, sizes, batch):
    torch = torch_cuda
    rng = np.random.default_rng(3)
    m, p = _mlp(sizes, batch)
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    out = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    _, ref = mo.forward(p.astype(np.float64), sizes, X.astype(np.float64))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out - ref)) <= 3e-2 * scale
    assert _cos(out.ravel(), ref.ravel()) >= 0.9995
    loss = m.backward(torch.from_numpy(T).cuda())
    ref_loss, ref_g = mo.loss_and_grad(p.astype(np.float64), sizes, X.astype(np.float64),
                                       T.astype(np.float64))
    assert loss == pytest.approx(ref_loss, rel=3e-2)
    g = m.get_grads().astype(np.float64)
    off = 0
    for l in range(len(sizes) - 1):
        nw = sizes[l + 1] * sizes[l]
        for a, b in ((off, off + nw), (off + nw, off + nw + sizes[l + 1])):
            assert _cos(g[a:b], ref_g[a:b]) >= 0.999, (l, a, b)
        off += nw + sizes[l + 1]
    m.close()


def test_adam_first_step(torch_cuda):
    torch = torch_cuda
    sizes, batch = [20, 32, 10], 16
    rng = np.random.default_rng(4)
    m, p = _mlp(sizes, batch)
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    m.forward(torch.from_numpy(X).cuda())
    m.backward(torch.from_numpy(T).cuda())
    g = m.get_grads()
    m.adam_step(lr=1e-3, step=1)
    p1 = m.get_params()
    # the first bias-corrected Adam step moves every parameter by lr * g/(|g| + eps)
    want = p - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, want, rtol=1e-5, atol=1e-7)
    _, ref_g = mo.loss_and_grad(p.astype(np.float64), sizes, X.astype(np.float64),
                                T.astype(np.float64))
    big = np.abs(ref_g) > 1e-2 * np.max(np.abs(ref_g))
    assert np.mean(np.sign(g[big]) == np.sign(ref_g[big])) >= 0.99
    m.close()


def test_warm_start_network_shape(torch_cuda):
    """The 10001 -> 512 -> 512 -> 5202 network at batch 256 (split-K on every GEMM)."""
    torch = torch_cuda
    sizes, batch = [10001, 512, 512, 5202], 256
    rng = np.random.default_rng(5)
    m, p = _mlp(sizes, batch)
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    out = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    _, ref = mo.forward(p.astype(np.float64), sizes, X.astype(np.float64))
    assert np.max(np.abs(out - ref)) <= 3e-2 * np.max(np.abs(ref))
    m.backward(torch.from_numpy(T).cuda())
    g = m.get_grads().astype(np.float64)
    _, ref_g = mo.loss_and_grad(p.astype(np.float64), sizes, X.astype(np.float64),
                                T.astype(np.float64))
    assert _cos(g, ref_g) >= 0.999
    m.close()


def test_training_reduces_loss(torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(6)
    sizes, batch = [12, 64, 64, 6], 64
    W = rng.standard_normal((6, 12))
    X = rng.standard_normal((batch, 12)).astype(np.float32)
    T = np.tanh(X @ W.T).astype(np.float32)
    m, _ = _mlp(sizes, batch)
    xt, tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    losses = []
    for step in range(1, 301):
        m.forward(xt)
        losses.append(m.backward(tt))
        m.adam_step(lr=3e-3, step=step)
    assert losses[-1] < 0.1 * losses[0]
    m.close()
