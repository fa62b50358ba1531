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
