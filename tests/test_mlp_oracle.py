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


# --------------------------------------------------------------------------
# BF16 reading: rounding points of the reduced-precision network
# --------------------------------------------------------------------------

def test_bf16_rounding_matches_library_conversion():
    """Round-to-nearest-even to BF16 against torch's own FP32 -> BF16
    conversion, plus the tie cases by hand (7 fraction bits: 1 + 2^-8 lies
    halfway between 1 and 1 + 2^-7 and goes to the even 1; 1 + 3 * 2^-8 goes
    to the even 1 + 2^-6)."""
    import torch
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = R.bf16(x)
    assert np.array_equal(got, ref)
    assert R.bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert R.bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert R.bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7


def test_bf16_mode_is_exact_on_representable_linear_layers():
    """One linear layer whose input, weights, bias and targets are BF16 values
    with short mantissas: every rounding point sees an exact value, so the BF16
    reading equals the FP64 network, output and gradients alike."""
    rng = np.random.default_rng(8)
    W = rng.integers(-8, 9, (5, 4)) / 8.0
    b = rng.integers(-8, 9, 4) / 16.0
    x = rng.integers(-4, 5, (6, 5)) / 4.0
    params = [(W, b)]
    # residuals 3k over 24 outputs: loss gradients 2 * 3k / 24 = k / 4, exact in BF16
    y = x @ W + b - rng.integers(-2, 3, (6, 4)) * 3.0
    o64, _, _ = R.forward(params, x)
    o16, _, _ = R.forward(params, x, bf16=True)
    assert np.array_equal(o64, o16)
    l64, g64 = R.backward(params, x, y)
    l16, g16 = R.backward(params, x, y, bf16=True)
    assert l64 == l16
    for (a, c), (d, e) in zip(g64, g16):
        assert np.array_equal(a, d) and np.array_equal(c, e)


def test_bf16_mode_rounds_hidden_activations():
    """Two layers: the BF16 reading feeds the second product with the rounded
    GELU of the first layer (checked against rounding it by hand)."""
    params = R.init_params((3, 8, 2), seed=9)
    x = np.random.default_rng(10).uniform(-1, 1, (5, 3))
    out, pres, acts = R.forward(params, x, bf16=True)
    h1 = R.bf16(R.gelu(R.bf16(x) @ R.bf16(params[0][0]) + params[0][1]))
    assert np.array_equal(acts[1], h1)
    assert np.array_equal(out, h1 @ R.bf16(params[1][0]) + params[1][1])
    # and it differs from the FP64 network by BF16 rounding only
    o64, _, _ = R.forward(params, x)
    assert 0 < np.max(np.abs(out - o64)) < 2.0 ** -5 * np.max(np.abs(o64))
