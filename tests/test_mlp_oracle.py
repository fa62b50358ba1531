"""Pins of the FP64 MLP oracle: central finite differences of its loss, the
closed form of one Adam step, and a linear network's normal equations."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo


@pytest.mark.parametrize("sizes", [[5, 7, 6, 3], [4, 3], [3, 9, 2]])
def test_gradient_matches_central_differences(sizes):
    rng = np.random.default_rng(0)
    p = rng.standard_normal(mo.num_params(sizes)) * 0.5
    X = rng.standard_normal((6, sizes[0]))
    T = rng.standard_normal((6, sizes[-1]))
    _, g = mo.loss_and_grad(p, sizes, X, T)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mo.loss_and_grad(p + e, sizes, X, T)[0] - mo.loss_and_grad(p - e, sizes, X, T)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(1)
    g = rng.standard_normal(50)
    th, m, v = mo.adam_step(np.zeros(50), g, np.zeros(50), np.zeros(50), 1e-3, 0.9, 0.999, 0.0, 1)
    np.testing.assert_allclose(th, -1e-3 * np.sign(g), rtol=1e-12)


def test_linear_network_zero_gradient_at_least_squares():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, 3))
    T = rng.standard_normal((40, 2))
    Xa = np.hstack([X, np.ones((40, 1))])
    sol = np.linalg.lstsq(Xa, T, rcond=None)[0]          # (4, 2)
    W, b = sol[:3].T, sol[3]
    p = np.concatenate([W.ravel(), b])
    _, g = mo.loss_and_grad(p, [3, 2], X, T)
    assert np.max(np.abs(g)) < 1e-12


def test_second_adam_step_hand_worked():
    """Step 2 of bias-corrected Adam in exact fractions.  With beta1 = 1/2, beta2 = 3/4,
    eps = 0 and gradients g1, g2: m-hat_2 = (beta1 g1 + g2) / (1 + beta1) and
    v-hat_2 = (beta2 g1^2 + g2^2) / (1 + beta2) = (3 g1^2 + 4 g2^2) / 7.
      (g1, g2) = (1, 1):   m-hat = 1,    v-hat = 1 -> step -lr
      (g1, g2) = (1, -1):  m-hat = -1/3, v-hat = 1 -> step +lr/3
      (g1, g2) = (2, -2):  m-hat = -2/3, v-hat = 4 -> step +lr/3 (scale invariance)
      (g1, g2) = (-3, 3):  m-hat = 1,    v-hat = 9 -> step -lr/3
    and step 1 moves every parameter by -lr sign(g1)."""
    lr = 0.125
    g1 = np.array([1.0, 1.0, 2.0, -3.0])
    g2 = np.array([1.0, -1.0, -2.0, 3.0])
    th0 = np.array([0.5, -0.25, 1.0, 2.0])
    m = v = np.zeros(4)
    th1, m, v = mo.adam_step(th0, g1, m, v, lr, 0.5, 0.75, 0.0, 1)
    np.testing.assert_array_equal(th1, th0 - lr * np.sign(g1))
    th2, m, v = mo.adam_step(th1, g2, m, v, lr, 0.5, 0.75, 0.0, 2)
    want = th1 + lr * np.array([-1.0, 1.0 / 3.0, 1.0 / 3.0, -1.0 / 3.0])
    np.testing.assert_allclose(th2, want, rtol=0, atol=1e-15)


def test_adam_matches_its_closed_form_over_five_steps():
    """The recursion against the explicit weighted sums it unrolls to:
    m_t = (1 - b1) sum_i b1^(t-i) g_i,  v_t = (1 - b2) sum_i b2^(t-i) g_i^2,
    theta_t = theta_{t-1} - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)."""
    rng = np.random.default_rng(7)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    gs = rng.standard_normal((5, 30))
    th = rng.standard_normal(30)
    ref = th.copy()
    m = v = np.zeros(30)
    for t in range(1, 6):
        th, m, v = mo.adam_step(th, gs[t - 1], m, v, lr, b1, b2, eps, t)
        w1 = np.array([(1 - b1) * b1 ** (t - i) for i in range(1, t + 1)])
        w2 = np.array([(1 - b2) * b2 ** (t - i) for i in range(1, t + 1)])
        mt = w1 @ gs[:t]
        vt = w2 @ gs[:t] ** 2
        ref = ref - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(th, ref, rtol=1e-13, atol=1e-15)


# ---- the BF16-operand model and its error bounds ----

def test_bf16_round_is_round_to_nearest_even():
    """Against torch's CPU float32 -> bfloat16 conversion (round to nearest, ties to even),
    on random values and on exact ties of both parities."""
    import torch
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    bits = rng.integers(0, 2 ** 31, 2000, dtype=np.uint64)
    ties = (((bits >> 16) << 16) | 0x8000).astype(np.uint32).view(np.float32)  # halfway cases
    ties = ties[np.isfinite(ties) & (np.abs(ties) > 1e-30)]
    for v in (x, ties, -ties):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(mo.bf16_round(v), want)
    # by hand: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 and rounds to the even 1;
    # 1 + 3 * 2^-8 rounds up to 1 + 2^-6
    np.testing.assert_array_equal(mo.bf16_round([1 + 2 ** -8, 1 + 3 * 2 ** -8]),
                                  [1.0, 1 + 2 ** -6])


@pytest.mark.parametrize("sizes", [[6, 5, 4, 4], [9, 3], [7, 11, 5]])
def test_bf16_model_without_rounding_is_the_plain_network(sizes):
    """With the operand rounding switched off the BF16-operand model is the plain FP64
    network: same output, loss and gradient (pins its data flow: operands, transposes,
    bias, ReLU mask and the loss coefficient), and its bounds are FP32 accumulation only
    (no undecided rounding)."""
    rng = np.random.default_rng(12)
    p = (rng.standard_normal(mo.num_params(sizes)) * 0.5).astype(np.float32)
    X = rng.standard_normal((8, sizes[0])).astype(np.float32)
    T = rng.standard_normal((8, sizes[-1])).astype(np.float32)
    r = mo.forward_backward_bf16(p, sizes, X, T, rnd=lambda a: np.asarray(a, np.float64))
    _, out = mo.forward(p.astype(np.float64), sizes, X.astype(np.float64))
    loss, g = mo.loss_and_grad(p.astype(np.float64), sizes, X.astype(np.float64),
                               T.astype(np.float64))
    np.testing.assert_allclose(r["out"], out, rtol=1e-13, atol=1e-13)
    assert r["loss"] == pytest.approx(loss, rel=1e-13)
    # the model forms dZ with the FP32 coefficient 2 / (B N), the plain network exactly
    coef32 = float(np.float32(2.0) / np.float32(8 * sizes[-1]))
    np.testing.assert_allclose(r["grad"], g * coef32 / (2.0 / (8 * sizes[-1])), rtol=1e-12,
                               atol=1e-14)


def _fp32_product(A, B, rng, splits):
    """A @ B.T accumulated in FP32 in a random order, split into `splits` partial sums
    that are added in order (as a split reduction does)."""
    K = A.shape[1]
    perm = rng.permutation(K)
    parts = np.array_split(perm, splits)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    total = None
    for idx in parts:
        acc = np.zeros((A.shape[0], B.shape[0]), np.float32)
        for k in idx:
            acc = acc + np.outer(A32[:, k], B32[:, k])  # BF16 products are exact in FP32
        total = acc if total is None else (total + acc).astype(np.float32)
    return total


def _emulate_fp32(params32, sizes, X32, T32, rng):
    """One FP32 evaluation of the library's arithmetic (BF16 operands, FP32 accumulation in
    random orders) in numpy: the thing the bounds must cover."""
    layers = mo.unpack(np.asarray(params32, np.float32).astype(np.float64), sizes)
    f32 = np.float32
    h = mo.bf16_round(X32).astype(f32)
    Hs, Wbs = [h], []
    _emulate_fp32.hidden = Hs
    for l, (W, b) in enumerate(layers):
        Wb = mo.bf16_round(W).astype(f32)
        Wbs.append(Wb)
        z = (_fp32_product(h, Wb, rng, 3) + b.astype(f32)).astype(f32)
        if l < len(layers) - 1:
            h = mo.bf16_round(np.maximum(z, f32(0))).astype(f32)
            Hs.append(h)
        else:
            out = z
    B, NO = out.shape
    d = (out - T32.astype(f32)).astype(f32)
    loss = float(np.sum(d.astype(np.float64) ** 2) / (B * NO))
    g = (f32(2.0) / (f32(B) * f32(NO)) * d).astype(f32)
    dzf, dzb = g, mo.bf16_round(g).astype(f32)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        gW = _fp32_product(dzb.T, Hs[l].T, rng, 2)
        order = rng.permutation(B)
        gb = np.zeros(dzf.shape[1], f32)
        for r in order:
            gb = (gb + dzf[r]).astype(f32)
        grads[l] = (gW, gb)
        if l > 0:
            dH = _fp32_product(dzb, Wbs[l].T, rng, 2)
            dz = np.where(Hs[l] > 0, dH, f32(0)).astype(f32)
            dzf, dzb = dz, mo.bf16_round(dz).astype(f32)
    flat = np.concatenate([np.concatenate([a.ravel(), c]) for a, c in grads]).astype(np.float64)
    return out.astype(np.float64), loss, flat


def _net(rng, sizes):
    return np.concatenate([np.concatenate([rng.uniform(-1, 1, sizes[l + 1] * sizes[l])
                                           * np.sqrt(3.0 / sizes[l]),
                                           rng.uniform(-.1, .1, sizes[l + 1])])
                           for l in range(len(sizes) - 1)]).astype(np.float32)


@pytest.mark.parametrize("sizes,batch,tight", [([300, 40], 48, 1e-4),
                                               ([300, 120, 40], 48, 2e-3),
                                               ([300, 120, 90, 40], 48, 2e-2),
                                               ([10001, 256, 24, 12], 64, None)])
def test_bf16_model_bounds_cover_fp32_evaluations(sizes, batch, tight):
    """FP32 evaluations in random summation orders (which round some hidden activations
    and some dZ entries to a different BF16 neighbour than the FP64 model does) stay within
    the model's per-element bounds for the output, the loss and every gradient entry.
    The bounds are not vacuous: without hidden layers they are FP32 accumulation error
    only; each hidden layer adds the possible one-unit BF16 jumps of its undecided
    roundings, so the output bound's median grows with depth (`tight`, relative to the
    output scale).  At a reduction length of 10001 the worst-case FP32 error of the first
    layer already spans BF16 rounding steps, so the bounds after two hidden layers are wide
    (no `tight`); there the case is kept because FP32 sums really do round activations to
    the other BF16 neighbour, which exercises the jump terms.  (Exact comparisons at that
    width use lattice data: test_bf16_model_exact_forward_on_lattice_data.)"""
    rng = np.random.default_rng(13)
    p = _net(rng, sizes)
    X = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    r = mo.forward_backward_bf16(p, sizes, X, T)
    if len(sizes) > 2:
        assert r["ambiguous"] > 0   # the case exercises the rounding-jump terms
    flips = 0
    for trial in range(3):
        out, loss, g = _emulate_fp32(p, sizes, X, T, np.random.default_rng(100 + trial))
        flips += sum(int(np.count_nonzero(a != b))
                     for a, b in zip(_emulate_fp32.hidden[1:], r["hidden"]))
        assert np.all(np.abs(out - r["out"]) <= r["e_out"])
        assert abs(loss - r["loss"]) <= r["e_loss"]
        assert np.all(np.abs(g - r["grad"]) <= r["e_grad"])
    if sizes[0] > 1000:
        # at this reduction length FP32 sums do land on the other side of BF16 rounding
        # boundaries: the jump terms of the bounds are exercised, not only the FP32 ones
        assert flips > 0
    if tight is not None:
        assert np.median(r["e_out"]) < tight * np.max(np.abs(r["out"]))


def test_adam_fp32_bound_covers_float32_steps():
    """Five Adam steps evaluated in numpy float32 (one rounding per operation, hyperparameters
    that are FP32 values) stay within the bounds propagated by adam_step_fp32_bound."""
    rng = np.random.default_rng(14)
    lr, b1, b2, eps = 2.0 ** -7, 0.875, 0.9375, 2.0 ** -20
    n = 5000
    th = rng.standard_normal(n).astype(np.float32)
    gs = (rng.standard_normal((5, n)) * np.exp(rng.uniform(-6, 2, (5, n)))).astype(np.float32)
    f = np.float32
    t32, m32, v32 = th.copy(), np.zeros(n, f), np.zeros(n, f)
    t64, m64, v64 = th.astype(np.float64), np.zeros(n), np.zeros(n)
    et, em, ev = np.zeros(n), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = gs[step - 1]
        c1, c2 = f(1) - f(b1) ** f(step), f(1) - f(b2) ** f(step)
        m32 = f(b1) * m32 + (f(1) - f(b1)) * g
        v32 = f(b2) * v32 + (f(1) - f(b2)) * g * g
        t32 = t32 - f(lr) * (m32 / c1) / (np.sqrt(v32 / c2) + f(eps))
        t64, m64, v64, et, em, ev = mo.adam_step_fp32_bound(
            t64, g.astype(np.float64), m64, v64, et, em, ev, lr, b1, b2, eps, step)
        assert np.all(np.abs(t32.astype(np.float64) - t64) <= et), step
        # and the bound stays a few FP32 units of the parameter scale
        assert np.max(et / (np.abs(t64) + lr)) < 5e-5


def test_bf16_model_exact_forward_on_lattice_data():
    """Integer inputs, weights, biases and targets whose forward sums stay below 2^24: every
    FP32 evaluation of the forward pass is exact in any order, so FP32 evaluations in random
    orders equal the model's output bit for bit (with the hidden BF16 roundings of the exact
    integer pre-activations, several of them ties), and the backward bounds still hold."""
    rng = np.random.default_rng(15)
    sizes = [3000, 64, 48, 16]
    X, T, p = lattice_problem(rng, sizes, 32)
    r = mo.forward_backward_bf16(p, sizes, X, T, exact_forward=True)
    assert any(np.any(h != np.rint(h)) or np.any(np.abs(h) > 256) for h in r["hidden"])
    for trial in range(2):
        out, loss, g = _emulate_fp32(p, sizes, X, T, np.random.default_rng(200 + trial))
        np.testing.assert_array_equal(out, r["out"])
        assert abs(loss - r["loss"]) <= r["e_loss"]
        assert np.all(np.abs(g - r["grad"]) <= r["e_grad"])


def lattice_problem(rng, sizes, batch, wmax=(7, 7, 1)):
    """Integer data for a ReLU network whose forward sums are exact in FP32: inputs in
    {-1, 0, 1} with 40 nonzeros per row, integer weights |w| <= wmax[l] and small integer
    biases.  Every pre-activation is an integer, each later layer reads BF16 roundings of
    integers (still integers), and the sums of absolute products stay below 2^24 (checked),
    so every partial sum in any order is an exactly representable integer."""
    X = np.zeros((batch, sizes[0]), np.float32)
    for b in range(batch):
        idx = rng.choice(sizes[0], size=min(40, sizes[0]), replace=False)
        X[b, idx] = rng.choice([-1.0, 1.0], size=idx.size)
    parts = []
    for l in range(len(sizes) - 1):
        w = wmax[min(l, len(wmax) - 1)]
        parts.append(rng.integers(-w, w + 1, sizes[l + 1] * sizes[l]).astype(np.float64))
        parts.append(rng.integers(0, 4, sizes[l + 1]).astype(np.float64))
    p = np.concatenate(parts).astype(np.float32)
    T = rng.integers(-50, 50, (batch, sizes[-1])).astype(np.float32)
    h = np.abs(mo.bf16_round(X))
    for l, (W, b) in enumerate(mo.unpack(p.astype(np.float64), sizes)):
        mag = h @ np.abs(W).T + np.abs(b)
        assert np.max(mag) < 2.0 ** 24
        h = mo.bf16_round(mag)
    return X, T, p
