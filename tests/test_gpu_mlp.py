"""GPU warm-start MLP (BF16 operands on MFMA, FP32 accumulation) against the oracle's
BF16-operand model (oracle/mlp_oracle.forward_backward_bf16): the same BF16 roundings
of the input, the weights, the hidden activations and dZ, computed in FP64, with a
per-element bound on what FP32 accumulation (any order, split reductions) can change,
including the one-unit BF16 jumps where a rounding or a ReLU mask is undecided.  Every
output, loss and gradient entry must lie within its bound.

On integer data whose forward sums are exactly representable in FP32 (lattice data)
the forward pass has no rounding freedom at all and must match the model bit for bit,
at the full warm-start network shape."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo
from tests.test_mlp_oracle import lattice_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    return torch


def _mlp(sizes, batch, p):
    from paper_2311_07710_amd.mlp import MLP
    m = MLP(sizes, max_batch=batch)
    m.set_params(p)
    return m


def _check_against_model(torch, sizes, X, T, p, exact_forward=False):
    m = _mlp(sizes, X.shape[0], p)
    out = m.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    loss = m.backward(torch.from_numpy(T).cuda())
    g = m.get_grads().astype(np.float64)
    m.close()
    r = mo.forward_backward_bf16(p, sizes, X, T, exact_forward=exact_forward)
    if exact_forward:
        np.testing.assert_array_equal(out, r["out"])
    else:
        bad = np.abs(out - r["out"]) > r["e_out"]
        assert not bad.any(), (np.argwhere(bad)[:5], out[bad][:5], r["out"][bad][:5])
    # the library reports the FP64 loss rounded to FP32
    assert abs(loss - r["loss"]) <= r["e_loss"] + 2 ** -23 * abs(r["loss"])
    bad = np.abs(g - r["grad"]) > r["e_grad"]
    assert not bad.any(), (np.flatnonzero(bad)[:5], g[bad][:5], r["grad"][bad][:5],
                           r["e_grad"][bad][:5])
    return out, g, r


@pytest.mark.parametrize("sizes,batch", [([37, 64, 48, 29], 50), ([8, 5], 3),
                                         ([100, 130, 70], 129), ([600, 40], 64),
                                         ([300, 96, 24], 32)])
def test_forward_backward_within_bf16_model_bounds(torch_cuda, sizes, batch):
    rng = np.random.default_rng(3)
    from paper_2311_07710_amd.mlp import init_params
    p = init_params(sizes, seed=0, out_scale=1.0)
    p[p == 0] = rng.uniform(-0.1, 0.1, np.count_nonzero(p == 0)).astype(np.float32)  # biases
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    out, g, r = _check_against_model(torch_cuda, sizes, X, T, p)
    # the bounds are FP32-accumulation sized where nothing is undecided: without hidden
    # layers the output bound is a small multiple of K u of the products' magnitude
    if len(sizes) == 2:
        assert np.median(r["e_out"]) < 1e-3 * np.max(np.abs(r["out"]))


def test_warm_start_shape_exact_forward(torch_cuda):
    """The 10001 -> 512 -> 512 -> 5202 network at batch 256 (split-K on every product) on
    lattice data: the forward output equals the model bit for bit (its hidden layer rounds
    thousands of integers to BF16), and the gradient is within the model's bounds."""
    sizes, batch = [10001, 512, 512, 5202], 256
    X, T, p = lattice_problem(np.random.default_rng(15), sizes, batch, wmax=(5, 1, 1))
    _check_against_model(torch_cuda, sizes, X, T, p, exact_forward=True)


def test_warm_start_shape_random_data(torch_cuda):
    """Realistic data at the warm-start shape.  There the rigorous bounds are wide (the
    FP32 error of a 10001-term sum may cross BF16 rounding boundaries anywhere), so this is
    a coarse check: outputs within 3e-2 of the output scale, gradient direction >= 0.999."""
    torch = torch_cuda
    from paper_2311_07710_amd.mlp import init_params
    sizes, batch = [10001, 512, 512, 5202], 256
    rng = np.random.default_rng(5)
    p = init_params(sizes, seed=0, out_scale=1.0)
    m = _mlp(sizes, batch, p)
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    out = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    _, ref = mo.forward(p.astype(np.float64), sizes, X.astype(np.float64))
    assert np.max(np.abs(out - ref)) <= 3e-2 * np.max(np.abs(ref))
    m.backward(torch.from_numpy(T).cuda())
    g = m.get_grads().astype(np.float64)
    _, ref_g = mo.loss_and_grad(p.astype(np.float64), sizes, X.astype(np.float64),
                                T.astype(np.float64))
    assert float(g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g))) >= 0.999
    m.close()


def test_adam_five_steps_within_fp32_bounds(torch_cuda):
    """Five Adam steps on gradients set from the host, element-wise against the oracle's
    Adam with FP32 error bounds (hyperparameters that are FP32 values)."""
    sizes = [20, 32, 10]
    n = mo.num_params(sizes)
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(n).astype(np.float32)
    gs = (rng.standard_normal((5, n)) * np.exp(rng.uniform(-6, 2, (5, n)))).astype(np.float32)
    lr, b1, b2, eps = 2.0 ** -7, 0.875, 0.9375, 2.0 ** -20
    m = _mlp(sizes, 4, p0)
    th, mm, vv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    et, em, ev = np.zeros(n), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        m.set_grads(gs[step - 1])
        m.adam_step(lr=lr, beta1=b1, beta2=b2, eps=eps, step=step)
        th, mm, vv, et, em, ev = mo.adam_step_fp32_bound(
            th, gs[step - 1].astype(np.float64), mm, vv, et, em, ev, lr, b1, b2, eps, step)
        got = m.get_params().astype(np.float64)
        bad = np.abs(got - th) > et
        assert not bad.any(), (step, np.flatnonzero(bad)[:5])
    m.close()


def test_rows_forms_match_gathered_batch(torch_cuda):
    """forward_rows / backward_rows on a resident data set give exactly what forward /
    backward give on the gathered minibatch; an out-of-range row index is an error."""
    torch = torch_cuda
    from paper_2311_07710_amd import QPError
    from paper_2311_07710_amd.mlp import init_params
    sizes, batch = [37, 64, 29], 50
    rng = np.random.default_rng(8)
    p = init_params(sizes, seed=2, out_scale=1.0)
    Xall = rng.standard_normal((300, sizes[0])).astype(np.float32)
    Tall = rng.standard_normal((300, sizes[-1])).astype(np.float32)
    rows = rng.choice(300, batch, replace=False).astype(np.int32)
    m1, m2 = _mlp(sizes, batch, p), _mlp(sizes, batch, p)
    o1 = m1.forward(torch.from_numpy(Xall[rows]).cuda()).cpu().numpy()
    l1 = m1.backward(torch.from_numpy(Tall[rows]).cuda())
    xa, ta, ri = (torch.from_numpy(Xall).cuda(), torch.from_numpy(Tall).cuda(),
                  torch.from_numpy(rows).cuda())
    o2 = m2.forward_rows(xa, ri).cpu().numpy()
    l2 = m2.backward_rows(ta, ri)
    np.testing.assert_array_equal(o1, o2)
    assert l1 == l2
    np.testing.assert_array_equal(m1.get_grads(), m2.get_grads())
    bad = torch.from_numpy(np.array([0, 300], np.int32)).cuda()
    with pytest.raises(QPError):
        m2.forward_rows(xa, bad)
    # the handle stays usable after the rejected call
    np.testing.assert_array_equal(m2.forward_rows(xa, ri).cpu().numpy(), o1)
    m1.close()
    m2.close()


def test_training_reduces_loss(torch_cuda):
    torch = torch_cuda
    from paper_2311_07710_amd.mlp import init_params
    rng = np.random.default_rng(6)
    sizes, batch = [12, 64, 64, 6], 64
    W = rng.standard_normal((6, 12))
    X = rng.standard_normal((batch, 12)).astype(np.float32)
    T = np.tanh(X @ W.T).astype(np.float32)
    m = _mlp(sizes, batch, init_params(sizes, seed=0, out_scale=1.0))
    xt, tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    losses = []
    for step in range(1, 301):
        m.forward(xt)
        losses.append(m.backward(tt))
        m.adam_step(lr=3e-3, step=step)
    assert losses[-1] < 0.1 * losses[0]
    m.close()
