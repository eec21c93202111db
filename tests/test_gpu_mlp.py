"""BF16 matrix-core surrogate network on the GPU against the FP64 NumPy
reference (oracle/mlp_oracle.py)."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as R

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflat(vec, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = vec[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, vec[o:o + b]))
        o += b
    return out


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02005_amd as pkg
    pkg.load_library()
    return pkg


def test_gemm_lane_layout_single_layer(P):
    """One linear layer: exact up to FP32 summation order on BF16 inputs."""
    import torch
    sizes = (40, 72)
    rng = np.random.default_rng(0)
    params = [(rng.standard_normal((40, 72)).astype(np.float32), rng.standard_normal(72).astype(np.float32))]
    note("case: linear 40 -> 72, 23 rows")
    net = P.Mlp(sizes, 64, flat(params))
    x = rng.standard_normal((23, 40)).astype(np.float32)
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    ref = bf16(x).astype(np.float64) @ bf16(params[0][0]).astype(np.float64) + params[0][1]
    assert np.max(np.abs(y - ref)) < 1e-4 * np.max(np.abs(ref))


def test_forward_and_gradients_match_oracle(P):
    import torch
    sizes = (3, 64, 64, 40)
    params = R.init_params(sizes, seed=1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (20, 3))
    y = rng.standard_normal((20, 40))
    note("case: 3 -> 64 -> 64 -> 40 GELU network, 20 rows")
    net = P.Mlp(sizes, 64, flat(params))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    out = net.forward(xt).cpu().numpy()
    ref, _, _ = R.forward(params, x)
    assert np.linalg.norm(out - ref) < 2e-2 * np.linalg.norm(ref)
    loss = net.gradients(xt, yt)
    loss_ref, grads_ref = R.backward(params, x, y)
    assert loss == pytest.approx(loss_ref, rel=2e-2)
    _, g = net.get_params()
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(unflat(g, sizes), grads_ref)):
        assert np.linalg.norm(gW - rW) < 3e-2 * np.linalg.norm(rW), li
        assert np.linalg.norm(gb - rb) < 3e-2 * np.linalg.norm(rb), li


def test_first_adam_step_closed_form(P):
    import torch
    sizes = (3, 32, 16)
    params = R.init_params(sizes, seed=3)
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.uniform(-1, 1, (16, 3)), dtype=torch.float32, device="cuda")
    y = torch.tensor(rng.standard_normal((16, 16)), dtype=torch.float32, device="cuda")
    net = P.Mlp(sizes, 64, flat(params))
    net.gradients(x, y)
    p0, g0 = net.get_params()
    net.train_step(x, y, 1e-3)
    net.sync()
    p1, _ = net.get_params()
    big = np.abs(g0) > 1e-4
    assert np.allclose((p1 - p0)[big], -1e-3 * np.sign(g0[big]), rtol=2e-3, atol=1e-6)
    assert np.all(np.abs((p1 - p0)[~big]) <= 1e-3 * (1 + 1e-6))


def test_training_tracks_oracle(P):
    import torch
    sizes = (3, 64, 64, 30)
    params = R.init_params(sizes, seed=5)
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (64, 3))
    y = np.tanh(x @ rng.standard_normal((3, 30)))
    net = P.Mlp(sizes, 64, flat(params))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    opt = R.Adam(params, lr=2e-3)
    ref = params
    for it in range(200):
        lg = net.train_step(xt, yt, 2e-3)
        lr_, gr = R.backward(ref, x, y)
        ref = opt.step(ref, gr)
        if it == 0:
            first = float(lg.item())
            assert first == pytest.approx(lr_, rel=3e-2)
    net.sync()
    final_gpu = net.gradients(xt, yt)
    final_ref = R.mse(R.forward(ref, x)[0], y)
    note(f"loss {first:.4e} -> {final_gpu:.4e} (FP64 reference {final_ref:.4e})")
    assert final_gpu < 0.1 * first
    assert final_gpu < 3.0 * final_ref + 1e-4


PROD = (3, 256, 256, 256, 256, 579)  # the warm-start network: 347 203 parameters


def excess(gpu, ref):
    """max over elements of |gpu - ref| / (|ref| + rms(ref))."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(ref * ref)))
    return float(np.max(np.abs(gpu - ref) / (np.abs(ref) + rms)))


# Element-wise bars.  Against the BF16 reading of the oracle (the same values
# rounded to BF16 at the same points, FP64 elsewhere) only two differences
# remain: FP32 against FP64 accumulation (about K 2^-24 of the summed
# magnitudes, ~1.5e-5 at K = 256) and the rare value whose FP32 and FP64
# forms round to neighbouring BF16 numbers, which moves that value by one BF16
# unit (2^-8 to 2^-7 of itself) and an output built from it by at most that
# much of its largest term: bar 2^-7.  Against the FP64 network the BF16
# rounding itself counts (up to about 4e-2 at this size, measured between the
# oracle's two readings): bar 2^-4.
BAR_BF16, BAR_FP64 = 2.0 ** -7, 2.0 ** -4


@pytest.mark.parametrize("seed", [11, 12])
def test_production_network_elementwise(P, seed):
    """3 -> 4 x 256 -> 579 at batch 64: forward outputs, loss and every
    layer's weight and bias gradients, element by element."""
    import torch
    params = R.init_params(PROD, seed=seed)
    p32 = flat(params)  # the FP32 master values the GPU holds
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in unflat(p32, PROD)]
    rng = np.random.default_rng(seed + 100)
    x = rng.uniform(-1, 1, (64, 3)).astype(np.float32)
    y = (0.5 * rng.standard_normal((64, PROD[-1]))).astype(np.float32)
    note(f"case: production network {PROD}, batch 64, seed {seed}")
    net = P.Mlp(PROD, 64, p32)
    xt = torch.tensor(x, device="cuda")
    yt = torch.tensor(y, device="cuda")
    out = net.forward(xt).cpu().numpy()
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    ref16 = R.forward(params, x64, bf16=True)[0]
    ref64 = R.forward(params, x64)[0]
    e16, e64 = excess(out, ref16), excess(out, ref64)
    note(f"  output: vs BF16 reading {e16:.3e}, vs FP64 {e64:.3e}")
    assert e16 <= BAR_BF16 and e64 <= BAR_FP64
    loss = net.gradients(xt, yt)
    l16, g16 = R.backward(params, x64, y64, bf16=True)
    l64, g64 = R.backward(params, x64, y64)
    note(f"  loss: gpu {loss:.6e} BF16 reading {l16:.6e} FP64 {l64:.6e}")
    assert abs(loss - l16) <= 1e-5 * l16
    _, g = net.get_params()
    for li, ((gW, gb), (aW, ab), (bW, bb)) in enumerate(zip(unflat(g, PROD), g16, g64)):
        ew16, eb16, ew64, eb64 = excess(gW, aW), excess(gb, ab), excess(gW, bW), excess(gb, bb)
        note(f"  layer {li}: dW {ew16:.3e} / {ew64:.3e}, db {eb16:.3e} / {eb64:.3e} (BF16 reading / FP64)")
        assert ew16 <= BAR_BF16 and eb16 <= BAR_BF16, li
        assert ew64 <= BAR_FP64 and eb64 <= BAR_FP64, li
