"""Pins of the oracle's three-direction approximate factorisation (CPU only):
diffusion implicit in x, y and z through (I - b L_x)(I - b L_y)(I - b L_z)
with b = alpha dt nu / 2 (the tridiagonal approximate factorisation of the
base solver, Sec. II).

  * the periodic line solves equal a dense solve of the circulant matrix;
  * pure diffusion of a neutral ion perturbation along x and of a
    unidirectional velocity perturbation u(y, z) (an exact Navier-Stokes
    solution: no convection, no pressure) is second order in time;
  * the scheme stays bounded at ten times the explicit diffusion limit,
    where the explicit x/z diffusion grows without bound;
  * laminar Couette flow stays exact (wall stress 1/Re).
"""
import math

import numpy as np
import pytest


@pytest.fixture(autouse=True)
def _one_thread(oracle_mod):
    oracle_mod.set_threads(1)
    yield
    oracle_mod.set_threads(8)


def _circulant(N, h, beta):
    A = np.eye(N) * (1 + 2 * beta / h ** 2)
    for i in range(N):
        A[i, (i + 1) % N] -= beta / h ** 2
        A[i, (i - 1) % N] -= beta / h ** 2
    return A


@pytest.mark.parametrize("d", [0, 1])
def test_periodic_line_solves_equal_dense_solves(oracle_mod, d):
    o = oracle_mod.Oracle(nx=12, ny=5, nz=6, implicit_xz=1)
    rng = np.random.default_rng(d)
    r = rng.standard_normal(o.shape)
    beta = 0.37
    out = o.xz_solve(d, beta, r)
    if d == 0:
        A = _circulant(o.nx, o.dx, beta)
        ref = np.einsum("ab,jkb->jka", np.linalg.inv(A), r)
    else:
        A = _circulant(o.nz, o.dz, beta)
        ref = np.einsum("ab,jbi->jai", np.linalg.inv(A), r)
    assert np.max(np.abs(out - ref)) < 1e-13


def _rest(oracle_mod, **kw):
    args = dict(nx=16, ny=9, nz=4, re=1.0, sc=1.0, debye=0.1, vhat=0.0, u_top=0.0, u_bot=0.0,
                stretch=1.0, implicit_xz=1)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    return o


def _ion_decay_error(oracle_mod, dt, T=0.24, implicit=1):
    o = _rest(oracle_mod, dt=dt, implicit_xz=implicit)
    x = (np.arange(o.nx) + 0.5) * o.dx
    prof = 1.0 + 0.1 * np.cos(2 * np.pi * x / o.cfg.lx)
    o.field("cp")[...] = prof[None, None, :]
    o.field("cm")[...] = prof[None, None, :]  # neutral: no charge, no potential
    o.solve_potential()
    o.run(int(round(T / dt)) * 3)
    k2 = (2 - 2 * math.cos(2 * math.pi * o.dx / o.cfg.lx)) / o.dx ** 2
    exact = 1.0 + 0.1 * np.cos(2 * np.pi * x / o.cfg.lx) * math.exp(-k2 * T)  # kd = 1/(Re Sc) = 1
    return np.max(np.abs(o.field("cp")[0, 0, :] - exact))


def test_ion_diffusion_in_x_is_second_order(oracle_mod):
    e1 = _ion_decay_error(oracle_mod, 0.04)
    e2 = _ion_decay_error(oracle_mod, 0.02)
    e3 = _ion_decay_error(oracle_mod, 0.01)
    assert 3.3 < e1 / e2 < 4.7 and 3.3 < e2 / e3 < 4.7, (e1, e2, e3)


def _shear_state(oracle_mod, dt, implicit=1):
    o = oracle_mod.Oracle(nx=4, ny=17, nz=16, re=2.0, debye=0.1, vhat=0.0, dt=dt, stretch=1.2,
                          implicit_xz=implicit)
    o.init(0, 0.0, 0.0)
    z = (np.arange(o.nz) + 0.5) * o.dz
    yc = o.yc
    pert = 0.2 * np.sin(2 * np.pi * z / o.cfg.lz)[None, :, None] * np.cos(0.5 * np.pi * yc)[:, None, None]
    o.field("u")[...] = yc[:, None, None] + pert
    return o


def test_unidirectional_velocity_decay_is_second_order(oracle_mod):
    T = 0.24
    ref = _shear_state(oracle_mod, 0.0025)
    ref.run(int(round(T / 0.0025)) * 3)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        o = _shear_state(oracle_mod, dt)
        o.run(int(round(T / dt)) * 3)
        assert np.max(np.abs(o.field("v"))) < 1e-13 and np.max(np.abs(o.field("p"))) < 1e-10
        errs.append(np.max(np.abs(o.field("u") - ref.field("u"))))
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_stable_beyond_the_explicit_diffusion_limit(oracle_mod):
    o = _rest(oracle_mod, dt=1.0)
    limit = 1.0 / (4 / o.dx ** 2 + 4 / o.dz ** 2)
    dt = 10 * limit
    growth = {}
    for imp in (1, 0):
        o = _rest(oracle_mod, dt=dt, implicit_xz=imp)
        rng = np.random.default_rng(1)
        noise = 1e-3 * rng.standard_normal(o.shape)
        o.field("cp")[...] = 1.0 + noise
        o.field("cm")[...] = 1.0 + noise
        o.solve_potential()
        o.run(60)
        growth[imp] = np.max(np.abs(o.field("cp") - 1.0)) / np.max(np.abs(noise))
    assert growth[1] < 1.0 and growth[0] > 1e3, growth


def test_laminar_couette_stays_exact(oracle_mod):
    o = oracle_mod.Oracle(nx=8, ny=17, nz=8, re=50.0, vhat=0.0, dt=0.02, implicit_xz=1)
    o.init(0, 0.0, 0.0)
    o.run(30)
    assert np.max(np.abs(o.field("u") - o.yc[:, None, None])) < 1e-13
    tb, tt = o.wall_shear()
    assert abs(tb - 1 / 50.0) < 1e-13 and abs(tt - 1 / 50.0) < 1e-13


def _noisy(oracle_mod, dt):
    o = oracle_mod.Oracle(nx=8, ny=9, nz=8, re=20.0, debye=0.2, vhat=2.0, dt=dt, stretch=1.2, implicit_xz=1)
    o.init(3, 0.1, 1e-2)
    return o


def test_velocity_with_pressure_converges_at_second_order(oracle_mod):
    """A noisy low-Re flow (projection active): the velocity converges at
    second order in time.  (The pressure of this fractional-step scheme is
    first order in time, with or without the implicit x/z part.)"""
    T = 0.12
    ref = _noisy(oracle_mod, 0.00125)
    ref.run(int(round(T / 0.00125)) * 3)
    e = []
    for dt in (0.02, 0.01, 0.005):
        o = _noisy(oracle_mod, dt)
        o.run(int(round(T / dt)) * 3)
        e.append(np.max(np.abs(o.field("u") - ref.field("u"))))
    assert 3.3 < e[0] / e[1] < 4.8 and 3.3 < e[1] / e[2] < 4.8, e


def _lxx(q, h):
    return (np.roll(q, -1, axis=2) - 2 * q + np.roll(q, 1, axis=2)) / h ** 2


def _lzz(q, h):
    return (np.roll(q, -1, axis=1) - 2 * q + np.roll(q, 1, axis=1)) / h ** 2


def _factorised_residual(oracle_mod, dt):
    """One substep against the factorised Crank-Nicolson momentum equation
    with the new pressure,
      (I - b Lx)(I - b Ly)(I - b Lz)(u1 - u0)
        = dt (gam H^k + zet H^{k-1}) - alpha dt G_x p1 + alpha dt nu (Lx + Ly + Lz) u0,
    b = alpha dt / (2 Re); interior rows.  With the pressure update
    p += psi - b (Lx + Ly + Lz) psi the residual is alpha dt F G psi with F
    the b^2 cross terms of the product, O(dt^4); an update with L_y alone
    leaves alpha dt b G (Lx + Lz) psi, O(dt^3)."""
    re = 20.0
    o = oracle_mod.Oracle(nx=8, ny=13, nz=8, re=re, debye=0.2, vhat=2.0, dt=dt, stretch=1.2, implicit_xz=1)
    o.init(3, 0.1, 1e-2)
    gam = [8 / 15, 5 / 12, 3 / 4]
    zet = [0.0, -17 / 60, -5 / 12]
    o.substep()  # now at stage 1: H^{k-1} is live
    k = o.stage
    a = gam[k] + zet[k]
    b = a * dt / (2 * re)
    u0, hold = o.field("u").copy(), o.hold(0).copy()
    h = o.explicit_terms()["u"]
    o.substep()
    u1, p1 = o.field("u").copy(), o.field("p").copy()
    gx = o.gradient(p1)[0]
    d = u1 - u0
    # apply the factorised operator: z, then y (zero wall values of the difference), then x
    t = d - b * _lzz(d, o.dz)
    t = t - b * o.apply_ly(t, 1, 0.0, 0.0)
    lhs = t - b * _lxx(t, o.dx)
    lap_u0 = o.apply_ly(u0, 1, -1.0, 1.0) + _lxx(u0, o.dx) + _lzz(u0, o.dz)
    rhs = dt * (gam[k] * h + zet[k] * hold) - a * dt * gx + a * dt / re * lap_u0
    return np.max(np.abs((lhs - rhs)[1:-1]))


def test_pressure_update_follows_the_factorised_operator(oracle_mod):
    r1 = _factorised_residual(oracle_mod, 0.02)
    r2 = _factorised_residual(oracle_mod, 0.01)
    assert r1 / r2 > 12.0, (r1, r2)
