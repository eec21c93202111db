"""Pins of the FP64 surrogate-network reference (CPU only): GELU against its
limits and derivative, analytic gradients against central finite
differences, the first Adam step against its closed form (every parameter
moves by lr * sign(g)), and a loss that decreases under training."""
import numpy as np
import pytest

from oracle import mlp_oracle as R


def test_parameter_count():
    # 3 -> 256 -> 256 -> 256 -> 256 -> 579
    assert R.param_count() == 347203


def test_gelu_limits_and_derivative():
    x = np.linspace(-8, 8, 1601)
    g = R.gelu(x)
    assert abs(R.gelu(np.array(0.0))) == 0.0
    assert np.allclose(g[x > 6], x[x > 6], atol=1e-8)
    assert np.allclose(g[x < -6], 0.0, atol=1e-8)
    assert R.gelu_grad(np.array(0.0)) == pytest.approx(0.5, abs=1e-15)
    h = 1e-6
    fd = (R.gelu(x + h) - R.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - R.gelu_grad(x))) < 1e-8
    # x Phi(x) with Phi the normal CDF: GELU(1) = Phi(1) = 0.8413447460685429
    assert R.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-14)


def test_gradients_match_finite_differences():
    sizes = (3, 7, 6, 5)
    params = R.init_params(sizes, seed=1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (4, 3))
    y = rng.standard_normal((4, 5))
    loss, grads = R.backward(params, x, y)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for q in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[q]
                flat[q] = old + h
                lp = R.mse(R.forward(params, x)[0], y)
                flat[q] = old - h
                lm = R.mse(R.forward(params, x)[0], y)
                flat[q] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[q]) < 1e-7 * max(1.0, abs(fd)), (li, q, fd, gflat[q])


def test_first_adam_step_moves_by_learning_rate():
    params = R.init_params((3, 4, 2), seed=3)
    rng = np.random.default_rng(4)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    opt = R.Adam(params, lr=1e-3)
    new = opt.step(params, grads)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W1 - W, -1e-3 * np.sign(gW), rtol=1e-4, atol=1e-12)
        assert np.allclose(b1 - b, -1e-3 * np.sign(gb), rtol=1e-4, atol=1e-12)


def test_training_reduces_loss():
    sizes = (3, 32, 32, 10)
    params = R.init_params(sizes, seed=5)
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (16, 3))
    y = np.sin(x @ rng.standard_normal((3, 10)))
    opt = R.Adam(params, lr=3e-3)
    l0, _ = R.backward(params, x, y)
    for _ in range(300):
        loss, grads = R.backward(params, x, y)
        params = opt.step(params, grads)
    assert loss < 0.05 * l0
