"""Pins of the float64 selector reference: analytic gradients against
central finite differences, closed forms of the network and of the first Adam
step, and feature values of matrices whose statistics are known exactly."""
import numpy as np
import pytest

from oracle import mlp
from tests import tiny


def _setup(K, B, seed):
    rs = np.random.RandomState(seed)
    P = rs.normal(scale=0.3, size=mlp.param_count(K))
    X = rs.normal(size=(B, 7))
    T = rs.normal(size=(B, K))
    norm = np.concatenate([rs.normal(size=7), rs.uniform(0.5, 2.0, 7)])
    return P, X, T, norm


@pytest.mark.parametrize("K,seed", [(3, 0), (12, 1), (1, 2)])
def test_gradient_matches_finite_differences(K, seed):
    P, X, T, norm = _setup(K, 9, seed)
    loss, g = mlp.loss_and_grad(P, K, X, T, norm)
    rs = np.random.RandomState(seed + 100)
    idx = rs.choice(len(P), size=60, replace=False)
    h = 1e-6
    for q in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[q] += h
        Pm[q] -= h
        fd = (mlp.loss_and_grad(Pp, K, X, T, norm)[0] - mlp.loss_and_grad(Pm, K, X, T, norm)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])


def test_zero_weights_output_bias_and_zero_hidden_gradient():
    K = 5
    P = np.zeros(mlp.param_count(K))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(P, K)
    b3[:] = np.arange(K)
    X = np.random.RandomState(3).normal(size=(4, 7))
    Y, _ = mlp.forward(P, K, X)
    assert np.array_equal(Y, np.tile(np.arange(K, dtype=float), (4, 1)))
    _, g = mlp.loss_and_grad(P, K, X, np.zeros((4, K)))
    W1g, b1g, W2g, b2g, W3g, b3g = mlp.unpack(g, K)
    # ReLU of zero pre-activations passes no gradient below the last layer
    assert not W1g.any() and not W2g.any() and not W3g.any()
    assert np.allclose(b3g, 2 * np.arange(K) / K)


def test_first_adam_step_moves_each_parameter_by_lr():
    rs = np.random.RandomState(4)
    P = rs.normal(size=50)
    g = rs.normal(size=50)
    lr = 0.01
    P1, m, v = mlp.adam(P, np.zeros(50), np.zeros(50), g, lr, 0.9, 0.999, 0.0, 1)
    # bias-corrected first step: m_hat = g, v_hat = g^2, so the step is lr*sign(g)
    assert np.allclose(P1, P - lr * np.sign(g), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_closed_forms():
    n = 100
    ident = (np.arange(n + 1), np.arange(n))
    f = mlp.features(*ident, n)
    assert f[0] == np.log2(n) and f[1] == np.log2(n + 1)
    assert f[2] == 1.0 and f[3] == 0.0 and f[4] == 1.0 and f[5] == 0.0
    assert f[6] == pytest.approx(1.0 / n)
    # every row full: degree m, variance 0, bandwidth n-1 (row 0 to column n-1)
    full = (np.arange(0, n * n + 1, n), np.tile(np.arange(n), n))
    f = mlp.features(*full, n)
    assert f[2] == n and f[3] == 0.0 and f[4] == np.log2(1 + n)
    assert f[5] == np.log2(n) and f[6] == 1.0
    # degrees 0 and 10 alternating: mean 5, variance 25, one row in two empty
    rs = np.random.RandomState(5)
    pos, crd, _ = tiny.csr(rs, 10, 10, 0.0, empty_rows=set(range(0, 10, 2)),
                           full_rows=set(range(1, 10, 2)))
    f = mlp.features(pos, crd, 10)
    assert f[2] == 5.0 and f[3] == np.log2(1 + 25.0) and f[6] == 1.0
