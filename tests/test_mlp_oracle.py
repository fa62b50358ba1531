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
