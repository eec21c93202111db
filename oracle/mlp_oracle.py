"""FP64 NumPy reference of the warm-start surrogate network.

TEST INFRASTRUCTURE ONLY: the GPU library's BF16 training and inference
kernels are checked against this module.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.

The network maps the control parameters of a plane-Couette electrolyte run
(Sec. II: Reynolds number, dimensionless voltage, Debye length) to its
mean wall-normal profiles: a fully connected perceptron with GELU hidden
activations (erf form, Hendrycks & Gimpel 2016), mean-squared-error loss and
the Adam optimiser (Kingma & Ba, ICLR 2015).  Layer l computes
y = x W_l + b_l with W_l of shape [in, out]; every hidden layer applies GELU.

Arithmetic: FP64 throughout by default.  With bf16=True the reference takes
the surrogate's reduced-precision reading (BF16 weights and activations, every
product accumulated in at least FP32): it rounds to BF16 (round to nearest,
ties to even, through FP32) exactly where that reading stores BF16 values --
the network input, every weight matrix, every hidden activation, the output
layer's loss gradient and every back-propagated pre-activation gradient --
and keeps everything else (accumulation, biases, the output, GELU and its
derivative) in FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    """x * Phi(x), Phi the standard normal distribution function."""
    return 0.5 * x * (1.0 + erf(x * SQRT1_2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x * SQRT1_2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def bf16(x):
    """Nearest BF16 value (ties to even) of each entry, via its FP32 value,
    returned as FP64.  BF16 keeps the sign, the 8 exponent bits and the top 7
    fraction bits of an FP32 number; the rounding adds half a unit of the
    kept part (minus one when the kept part is even, for ties to even) to the
    32-bit pattern and truncates the low 16 bits."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rnd(x, on):
    return bf16(x) if on else x


def init_params(sizes, seed=0):
    """He-style uniform initialisation, weights [in, out], zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        bound = math.sqrt(6.0 / fin)
        params.append((rng.uniform(-bound, bound, (fin, fout)), np.zeros(fout)))
    return params


def forward(params, x, bf16=False):
    """Returns the output and the per-layer pre-activations and inputs (the
    inputs as the products see them: BF16-rounded when bf16 is set)."""
    h = _rnd(x, bf16)
    acts = [h]
    pres = []
    for li, (W, b) in enumerate(params):
        z = h @ _rnd(W, bf16) + b
        pres.append(z)
        h = _rnd(gelu(z), bf16) if li < len(params) - 1 else z
        acts.append(h)
    return h, pres, acts


def mse(yhat, y):
    """mean over samples and outputs of (yhat - y)^2."""
    return float(np.mean((yhat - y) ** 2))


def backward(params, x, y, bf16=False):
    """Loss and its gradient with respect to every W and b (chain rule).
    With bf16 set, the gradient of each pre-activation is rounded to BF16
    once formed (the loss gradient at the output, (g W^T) * GELU'(z) below)."""
    yhat, pres, acts = forward(params, x, bf16)
    loss = mse(yhat, y)
    g = _rnd(2.0 * (yhat - y) / yhat.size, bf16)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (acts[li].T @ g, g.sum(axis=0))
        if li > 0:
            g = _rnd((g @ _rnd(W, bf16).T) * gelu_grad(pres[li - 1]), bf16)
    return loss, grads


class Adam:
    """m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for q, (p, gq) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[li][q] + (1 - self.b1) * gq
                v = self.b2 * self.v[li][q] + (1 - self.b2) * gq * gq
                self.m[li] = tuple(m if r == q else self.m[li][r] for r in range(2))
                self.v[li] = tuple(v if r == q else self.v[li][r] for r in range(2))
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append(tuple(new))
        return out


SIZES = (3, 256, 256, 256, 256, 579)


def param_count(sizes=SIZES):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))
