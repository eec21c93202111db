"""Pins of the oracle's building blocks against library routines, brute force
and published values.  These run on the CPU only.

The elliptic solver of the paper (Sec. II) is a Fourier transform in the two
periodic directions plus a Thomas solve across the gap; the oracle implements
both itself, so both are checked here against independent references.
"""
from pathlib import Path

import numpy as np
import pytest
from scipy.linalg import solve_banded

GOLDEN = Path(__file__).resolve().parent / "golden"


def test_splitmix64_published_vector(oracle_mod):
    """The seeded-noise generator is SplitMix64; its published test vector."""
    rows = [int(x) for x in (GOLDEN / "splitmix64_seed1234567.txt").read_text().split("\n")
            if x.strip() and not x.startswith("#")]
    got = [oracle_mod.splitmix_raw(1234567, n) for n in range(1, 6)]
    assert got == rows


def test_noise_is_uniform_and_field_dependent(oracle_mod):
    vals = np.array([oracle_mod.noise(7, 0, i) for i in range(20000)])
    assert vals.min() >= -1.0 and vals.max() < 1.0
    assert abs(vals.mean()) < 0.02
    assert abs(vals.var() - 1.0 / 3.0) < 0.01
    other = np.array([oracle_mod.noise(7, 1, i) for i in range(2000)])
    assert abs(np.corrcoef(vals[:2000], other)[0, 1]) < 0.08


SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64, 96, 128, 256, 384, 512]


@pytest.mark.parametrize("n", SIZES)
def test_fft_matches_numpy(oracle_mod, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = oracle_mod.fft(x, -1)
    ref = np.fft.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    inv = oracle_mod.fft(x, +1)
    ref_inv = np.fft.ifft(x) * n
    assert np.max(np.abs(inv - ref_inv)) <= 1e-13 * max(1.0, np.max(np.abs(ref_inv)))


@pytest.mark.parametrize("n", [3, 12, 48, 64])
def test_fft_matches_direct_dft(oracle_mod, n):
    """Brute-force O(N^2) DFT as an independent definition."""
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    k = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(k, k) / n)
    assert np.allclose(oracle_mod.fft(x, -1), W @ x, rtol=0, atol=1e-12 * np.abs(x).sum())


@pytest.mark.parametrize("n", [1, 2, 5, 64, 383])
def test_thomas_matches_banded_solver(oracle_mod, n):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = 2.5 + rng.uniform(0, 1, n)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ab = np.zeros((3, n))
    ab[0, 1:] = c[:-1]
    ab[1] = b
    ab[2, :-1] = a[1:]
    ref = solve_banded((1, 1), ab.astype(complex), d)
    got = oracle_mod.thomas(a, b, c, d)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_grid_is_tanh_stretched(oracle_mod):
    """y nodes tanh(g xi)/tanh(g) on xi uniform in [-1, 1]; centres midway."""
    o = oracle_mod.Oracle(nx=4, ny=33, nz=4, stretch=1.5)
    xi = -1 + 2 * np.arange(33) / 32
    assert np.allclose(o.yn, np.tanh(1.5 * xi) / np.tanh(1.5), atol=1e-15)
    assert np.allclose(o.yc, 0.5 * (o.yn[1:] + o.yn[:-1]), atol=1e-15)
    assert np.allclose(o.dn, np.diff(o.yn), atol=1e-15)
    dc = o.dc
    assert np.isclose(dc[0], o.dn[0] / 2) and np.isclose(dc[-1], o.dn[-1] / 2)
    assert np.allclose(dc[1:-1], np.diff(o.yc), atol=1e-15)
    # smallest spacing at the small config quoted as 2.04e-2
    assert abs(o.dn.min() - 2.04e-2) < 5e-4
    # dy/dxi is proportional to sech^2(g xi): spacing ratio -> cosh^2(g) = 5.53
    fine = oracle_mod.Oracle(nx=1, ny=1025, nz=1, stretch=1.5)
    assert fine.dn.max() / fine.dn.min() == pytest.approx(np.cosh(1.5) ** 2, rel=1e-2)


def test_coulomb_coupling_constant(oracle_mod):
    """K = beta/(2 Sc Re^2 lam^2); 1.5625e-4 at Re=400, lam=0.1, beta=0.5, Sc=1."""
    assert oracle_mod.coulomb_k(re=400, sc=1, beta=0.5, debye=0.1) == pytest.approx(1.5625e-4, rel=1e-14)
    assert oracle_mod.coulomb_k(re=3000, sc=3, beta=0.5, debye=0.01) == pytest.approx(
        0.5 / (2 * 3 * 3000.0 ** 2 * 1e-4), rel=1e-14)
