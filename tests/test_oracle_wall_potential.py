"""Pins of the oracle's arbitrary wall potential (CPU only): phi with given
wall values g(x, z) on the walls (beyond the uniform -+vhat/2 carried by
Phi_0), the inhomogeneous Dirichlet problem of the potential equation
(Sec. II).

  * uniform wall values -c / +c and no charge: the finite-volume operator
    with the wall value at the half-cell distance is exact for linear
    profiles, so phi = c y at every cell centre;
  * a wall pattern A cos(a x) cos(b z) on the lower wall and no charge: the
    discrete solution converges at second order in y to
    A cos(a x) cos(b z) sinh(K (1 - y)) / sinh(2 K), with K^2 the modified
    wavenumbers of the three-point x and z operators;
  * the problem is linear: charge and wall data superpose.
"""
import math

import numpy as np
import pytest


@pytest.fixture(autouse=True)
def _one_thread(oracle_mod):
    oracle_mod.set_threads(1)
    yield
    oracle_mod.set_threads(8)


def _uncharged(oracle_mod, nx=8, ny=33, nz=4, **kw):
    args = dict(nx=nx, ny=ny, nz=nz, re=100.0, debye=0.1, vhat=0.0, dt=1e-3, stretch=1.5)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    o.field("cp")[...] = 1.0
    o.field("cm")[...] = 1.0
    return o


def _xz(o):
    x = (np.arange(o.nx) + 0.5) * o.dx
    z = (np.arange(o.nz) + 0.5) * o.dz
    return x, z


def test_uniform_wall_values_give_a_linear_potential(oracle_mod):
    o = _uncharged(oracle_mod)
    c = 0.7
    o.set_wall_potential(np.full((o.nz, o.nx), -c), np.full((o.nz, o.nx), c))
    o.solve_potential()
    phi = o.field("phi")
    ref = c * o.yc[:, None, None]
    assert np.max(np.abs(phi - ref)) < 1e-12
    # cleared walls give back the homogeneous problem (zero without charge)
    o.set_wall_potential(None, None)
    o.solve_potential()
    assert np.max(np.abs(o.field("phi"))) < 1e-14


def test_wall_pattern_converges_at_second_order(oracle_mod):
    A, ma, mb = 0.5, 1, 1
    errs = []
    for ny in (17, 33, 65):
        o = _uncharged(oracle_mod, ny=ny, stretch=1.2)
        x, z = _xz(o)
        a = 2 * math.pi * ma / o.cfg.lx
        b = 2 * math.pi * mb / o.cfg.lz
        kx2 = (2 - 2 * math.cos(a * o.dx)) / o.dx ** 2
        kz2 = (2 - 2 * math.cos(b * o.dz)) / o.dz ** 2
        K = math.sqrt(kx2 + kz2)
        g = A * np.cos(b * z)[:, None] * np.cos(a * x)[None, :]
        o.set_wall_potential(g, None)
        o.solve_potential()
        yc = o.yc
        ref = g[None, :, :] * (np.sinh(K * (1 - yc)) / np.sinh(2 * K))[:, None, None]
        errs.append(np.max(np.abs(o.field("phi") - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, errs
    assert errs[-1] < 2e-4


def test_charge_and_wall_data_superpose(oracle_mod):
    rng = np.random.default_rng(4)
    o = _uncharged(oracle_mod, ny=17)
    dc = 0.01 * rng.standard_normal(o.shape)
    gb = 0.3 * rng.standard_normal((o.nz, o.nx))
    gt = 0.3 * rng.standard_normal((o.nz, o.nx))
    o.field("cp")[...] = 1.0 + dc
    o.solve_potential()
    only_charge = o.field("phi").copy()
    o.set_wall_potential(gb, gt)
    o.solve_potential()
    both = o.field("phi").copy()
    o.field("cp")[...] = 1.0
    o.solve_potential()
    only_wall = o.field("phi").copy()
    assert np.max(np.abs(both - only_charge - only_wall)) < 1e-13 * max(np.max(np.abs(both)), 1.0)
    assert np.max(np.abs(only_wall)) > 0.05
