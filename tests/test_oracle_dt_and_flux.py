"""Pins of the oracle's adaptive time-step rule and of the advective part of
its plane-averaged ion flux (CPU only).

Time step (reading of Sec. II: the explicit terms are advanced by the
three-stage Runge-Kutta scheme under a CFL condition; explicit migration adds
the Debye charge-relaxation limit and explicit horizontal diffusion its own
stability limit):
    dt = min( cfl / max_cells(|u_c|/dx + |v_c|/dy_j + |w_c|/dz),
              2 lam^2 Re Sc / max(c+ + c-),
              min(Re, Re Sc) / (4/dx^2 + 4/dz^2) )       (last term dropped
                                                            when x/z diffusion
                                                            is implicit)
with velocities averaged to the cell centres.  Each test below builds fields
for which one limit binds and its value follows by hand from the fields
(uniform velocities, a single concentration bump, a quiescent fluid), so a
wrong factor, a wrong spacing (node distance instead of cell height) or a
wrong viscosity in any limit fails.

Ion flux (Fig. 1 caption: the total wall-normal ion flux vanishes on the
walls): with uniform concentration c0, no potential perturbation and a wall
normal velocity whose plane mean is V1, the plane-averaged total flux of
species z at every interior node is c0 V1 (advection) minus
(Re Sc)^-1 z c0 vhat/2 (migration in the applied field), and exactly 0 on the
two walls.
"""
import numpy as np
import pytest


@pytest.fixture(autouse=True)
def _few_threads(oracle_mod):
    oracle_mod.set_threads(2)
    yield
    oracle_mod.set_threads(8)


def _tanh_nodes(ny, g):
    xi = -1.0 + 2.0 * np.arange(ny) / (ny - 1)
    return np.tanh(g * xi) / np.tanh(g)


def _state(oracle_mod, **kw):
    args = dict(nx=32, ny=33, nz=32, dt=0.0, cfl=0.5, stretch=1.5, vhat=0.0)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    for name in ("u", "v", "w", "phi", "p"):
        o.field(name)[...] = 0.0
    o.field("cp")[...] = 1.0
    o.field("cm")[...] = 1.0
    return o


def test_cfl_limit_with_uniform_horizontal_velocity(oracle_mod):
    """u = U0, w = W0 everywhere: rate = U0/dx + W0/dz in every cell."""
    o = _state(oracle_mod, re=1e6, debye=1.0)
    U0, W0 = 1.7, -0.6
    o.field("u")[...] = U0
    o.field("w")[...] = W0
    dx, dz = 2 * np.pi / 32, np.pi / 32
    expect = 0.5 / (U0 / dx + abs(W0) / dz)
    assert o.compute_dt() == pytest.approx(expect, rel=1e-14, abs=0)


def test_cfl_limit_uses_the_cell_height(oracle_mod):
    """v = V0 on every interior node (0 on the wall nodes): the centre value is
    V0 in rows 1 .. M-2 and V0/2 in the two wall rows, so with tanh clustering
    (second cell less than twice the first) the rate peaks in row 1 at
    V0 / (yn_2 - yn_1); adding u = U0 adds U0/dx to every cell."""
    ny = 33
    o = _state(oracle_mod, re=1e6, debye=1.0)
    V0, U0 = 0.3, 0.8
    o.field("v")[1:, :, :] = V0
    o.field("u")[...] = U0
    yn = _tanh_nodes(ny, 1.5)
    h0, h1 = yn[1] - yn[0], yn[2] - yn[1]
    assert h1 < 2 * h0  # the second row binds, not the first
    dx = 2 * np.pi / 32
    expect = 0.5 / (U0 / dx + V0 / h1)
    assert o.compute_dt() == pytest.approx(expect, rel=1e-14, abs=0)
    # a node-distance reading (centre-to-centre spacing) would give another value
    hc1 = 0.5 * (yn[3] + yn[2]) - 0.5 * (yn[2] + yn[1])
    assert abs(0.5 / (U0 / dx + V0 / hc1) - expect) > 1e-6 * expect


def test_cfl_limit_scales_with_cfl_number(oracle_mod):
    o1 = _state(oracle_mod, re=1e6, debye=1.0, cfl=0.5)
    o2 = _state(oracle_mod, re=1e6, debye=1.0, cfl=0.125)
    for o in (o1, o2):
        o.field("u")[...] = 1.0
    assert o2.compute_dt() == pytest.approx(0.25 * o1.compute_dt(), rel=1e-15)


def test_debye_relaxation_limit(oracle_mod):
    """Quiescent fluid, c+ = 3 in one cell and 1 elsewhere, c- = 1:
    max(c+ + c-) = 4, so dt = 2 lam^2 Re Sc / 4."""
    re, sc, lam = 1e4, 2.0, 0.01
    o = _state(oracle_mod, re=re, sc=sc, debye=lam)
    o.field("cp")[5, 7, 11] = 3.0
    expect = 2.0 * lam * lam * re * sc / 4.0
    # the other limits are far away: no CFL rate, diffusion limit >> expect
    dx, dz = 2 * np.pi / 32, np.pi / 32
    assert min(re, re * sc) / (4 / dx ** 2 + 4 / dz ** 2) > 10 * expect
    assert o.compute_dt() == pytest.approx(expect, rel=1e-14, abs=0)


@pytest.mark.parametrize("sc", [0.5, 3.0])
def test_horizontal_diffusion_limit(oracle_mod, sc):
    """Quiescent fluid with uniform ions: dt = min(Re, Re Sc)/(4/dx^2 + 4/dz^2)
    (the ions diffuse faster than momentum when Sc < 1)."""
    re, lam = 10.0, 1.0
    o = _state(oracle_mod, re=re, sc=sc, debye=lam, nx=24, nz=18, lx=3.0, lz=1.5)
    dx, dz = 3.0 / 24, 1.5 / 18
    expect = min(re, re * sc) / (4.0 / dx ** 2 + 4.0 / dz ** 2)
    assert 2.0 * lam * lam * re * sc / 2.0 > 10 * expect
    assert o.compute_dt() == pytest.approx(expect, rel=1e-14, abs=0)


def test_implicit_horizontal_diffusion_drops_its_limit(oracle_mod):
    """With x/z diffusion implicit the same quiescent state is limited by the
    Debye relaxation only."""
    re, sc, lam = 10.0, 0.5, 1.0
    o = _state(oracle_mod, re=re, sc=sc, debye=lam, implicit_xz=1)
    assert o.compute_dt() == pytest.approx(2.0 * lam * lam * re * sc / 2.0, rel=1e-14, abs=0)


def test_smallest_limit_wins(oracle_mod):
    """Uniform u with a concentration bump: the CFL and Debye values computed
    by hand; the rule returns the smaller, whichever it is."""
    dx = 2 * np.pi / 32
    for U0, bump in ((1.0, 1.0), (50.0, 1.0), (1.0, 400.0)):
        o = _state(oracle_mod, re=1e6, sc=1.0, debye=0.02)
        o.field("u")[...] = U0
        o.field("cm")[3, 4, 5] = bump
        cfl = 0.5 / (U0 / dx)
        deb = 2.0 * 0.02 ** 2 * 1e6 / (1.0 + bump)
        assert o.compute_dt() == pytest.approx(min(cfl, deb), rel=1e-14, abs=0)


def test_run_uses_the_rule_at_the_first_stage_only(oracle_mod):
    """An adaptive run sets dt from the rule at stage 1 and keeps it for the
    other two stages of the step."""
    o = oracle_mod.Oracle(nx=16, ny=17, nz=8, dt=0.0, cfl=0.5, re=300.0, vhat=3.0, debye=0.2)
    o.init(7, 0.05, 1e-3)
    d0 = o.compute_dt()
    o.substep()
    assert o.dt == d0
    o.substep()
    o.substep()
    assert o.dt == d0
    d1 = o.compute_dt()
    o.substep()
    assert o.dt == d1


@pytest.mark.parametrize("vhat", [0.0, 6.0])
def test_ion_flux_advection_and_applied_field(oracle_mod, vhat):
    """Uniform c0, phi = 0, v = V1 + A cos(2 pi x / Lx) on interior nodes:
    plane-mean flux of species z = c0 V1 - (Re Sc)^-1 z c0 vhat / 2 at
    interior nodes, 0 on the walls; ion contents c0 * (Lx * 2 * Lz)."""
    re, sc, c0, V1, A = 50.0, 2.0, 1.3, 0.07, 0.4
    nx, nz, ny = 16, 8, 17
    o = _state(oracle_mod, nx=nx, nz=nz, ny=ny, re=re, sc=sc, vhat=vhat)
    o.field("cp")[...] = c0
    o.field("cm")[...] = c0
    x = np.arange(nx) * (2 * np.pi / nx)
    o.field("v")[1:, :, :] = V1 + A * np.cos(x)[None, None, :]
    jp, jm, mp, mm = o.ion_flux()
    kd = 1.0 / (re * sc)
    assert jp[0] == 0.0 and jp[-1] == 0.0 and jm[0] == 0.0 and jm[-1] == 0.0
    np.testing.assert_allclose(jp[1:-1], c0 * V1 - kd * c0 * vhat / 2, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(jm[1:-1], c0 * V1 + kd * c0 * vhat / 2, rtol=1e-13, atol=1e-15)
    vol = 2 * np.pi * 2.0 * np.pi
    assert mp == pytest.approx(c0 * vol, rel=1e-13) and mm == pytest.approx(c0 * vol, rel=1e-13)


def test_ion_flux_of_a_linear_profile(oracle_mod):
    """Quiescent fluid, no field, c = a + b y at the cell centres: the
    plane-mean diffusive flux at node j is -(Re Sc)^-1 b (the centre
    difference of a linear profile is exact on any grid); with v = V1 the
    advective flux is V1 times the mean of the two adjacent centre values."""
    re, sc, a, b, V1 = 40.0, 1.0, 1.0, 0.25, -0.03
    o = _state(oracle_mod, nx=8, nz=4, ny=21, re=re, sc=sc)
    yc = o.yc
    o.field("cp")[...] = (a + b * yc)[:, None, None]
    o.field("cm")[...] = (a - b * yc)[:, None, None]
    o.field("v")[1:, :, :] = V1
    jp, jm, _, _ = o.ion_flux()
    kd = 1.0 / (re * sc)
    cf = a + b * 0.5 * (yc[1:] + yc[:-1])
    np.testing.assert_allclose(jp[1:-1], V1 * cf - kd * b, rtol=1e-12, atol=1e-15)
    cfm = a - b * 0.5 * (yc[1:] + yc[:-1])
    np.testing.assert_allclose(jm[1:-1], V1 * cfm + kd * b, rtol=1e-12, atol=1e-15)
