"""Pins of the limited advective face value of the ions (CPU only).

Sec. II discretises the advective flux with second-order central
differences: the face value of c is the mean of the two cells.  At the ions'
cell Peclet numbers in a turbulent run (Re Sc |u| h of order 10^2) the mean
lets a transported profile overshoot and undershoot, and steep near-wall
layers go negative.  Configuration migration_face = 2 (the hybrid migration
rule, plus this) takes the upwind cell of the face velocity and adds a van
Leer slope, which is the mean on a linear profile of equal spacings and the
upwind value at an extremum.  Pinned here by what the mathematics fixes,
not by retyping the face formula:
  * a square wave carried once around a periodic box, and a blob stirred by a
    2-D cellular flow between the walls, stay within their initial bounds,
    where the central form overshoots (and goes negative in the stirred case);
  * a sine carried by a uniform flow converges at second order to the exact
    translated, diffused wave;
  * where the profile is linear over the stencil, the explicit term equals
    the central one;
  * mirroring the profile and reversing the velocity mirrors the result
    (the upwind side is chosen by the velocity's sign), and the z direction
    gives the x direction's result with the axes exchanged;
  * the plane mean of the explicit ion term is minus the divergence of the
    plane-averaged advective and migration flux (update and flux diagnostic
    take the same face values, wall rows included), and mass is conserved.
"""
import numpy as np
import pytest


@pytest.fixture(autouse=True)
def _few_threads(oracle_mod):
    oracle_mod.set_threads(2)
    yield
    oracle_mod.set_threads(8)


def _passive(oracle_mod, face, **kw):
    """Uncharged passive ions: vhat = 0 and c+ = c- keep rho = 0 and Phi = 0,
    so both species obey the same advection-diffusion equation."""
    args = dict(nx=64, ny=5, nz=4, re=1e4, sc=10.0, debye=0.1, vhat=0.0, beta=0.0, u_top=1.0, u_bot=1.0,
                dt=0.0, cfl=0.5, migration_face=face)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    for n in ("u", "v", "w", "phi", "p"):
        o.field(n)[...] = 0.0
    return o


def _set_ions(o, c):
    for n in ("cp", "cm"):
        o.field(n)[...] = c


def test_square_wave_keeps_its_bounds(oracle_mod):
    lows, highs = {}, {}
    for face in (1, 2):
        o = _passive(oracle_mod, face)
        L = o.cfg.nx * o.dx
        x = (np.arange(o.cfg.nx) + 0.5) * o.dx
        _set_ions(o, np.where((x > 0.25 * L) & (x < 0.6 * L), 1.5, 0.5)[None, None, :])
        o.field("u")[...] = 1.0
        while o.t < L:  # once around the box at CFL 0.5
            o.run(20)
        lows[face], highs[face] = o.field("cp").min(), o.field("cp").max()
        np.testing.assert_array_equal(o.field("cp"), o.field("cm"))
    assert lows[2] >= 0.5 - 1e-13 and highs[2] <= 1.5 + 1e-13
    assert lows[1] < 0.4 and highs[1] > 1.6  # the central form's oscillations


def _cellular(oracle_mod, face, axis):
    """A blob in a 2-D cellular flow between the walls, in the x-y plane
    (axis 'x') or the z-y plane (axis 'z').  The initial velocity comes from a
    stream function at the cell corners, so its discrete divergence is zero;
    it then evolves under the momentum equations."""
    n_h, n_o = 32, 4
    l_h, l_o = 2 * np.pi, 1.0
    kw = dict(nx=n_h, nz=n_o, lx=l_h, lz=l_o) if axis == "x" else dict(nx=n_o, nz=n_h, lx=l_o, lz=l_h)
    o = _passive(oracle_mod, face, ny=33, re=1e3, u_top=0.0, u_bot=0.0, **kw)
    M = o.M
    h = o.dx if axis == "x" else o.dz
    L = n_h * h
    xf = np.arange(n_h) * h
    psi = np.sin(2 * np.pi * xf / L)[None, :] * np.sin(np.pi * (o.yn[:, None] + 1) / 2)  # [node][face]
    along = (psi[1:] - psi[:-1]) / o.dn[:, None]
    normal = -(np.roll(psi, -1, axis=1) - psi) / h
    xc = (np.arange(n_h) + 0.5) * h
    c = np.where((np.abs(xc - L / 2)[None, :] < L / 4) & (np.abs(o.yc)[:, None] < 0.4), 1.5, 0.5)
    if axis == "x":
        o.field("u")[...] = along[:, None, :]
        o.field("v")[...] = normal[:M][:, None, :]
        _set_ions(o, c[:, None, :])
    else:
        o.field("w")[...] = along[:, :, None]
        o.field("v")[...] = normal[:M][:, :, None]
        _set_ions(o, c[:, :, None])
    assert o.max_divergence() < 1e-13
    return o


def test_stirred_blob_keeps_its_bounds_and_mass(oracle_mod):
    lows = {}
    for face in (1, 2):
        o = _cellular(oracle_mod, face, "x")
        _, _, m0, _ = o.ion_flux()
        lo, hi = np.inf, -np.inf
        while o.t < 3.0:
            o.run(10)
            lo, hi = min(lo, o.field("cp").min()), max(hi, o.field("cp").max())
        _, _, m1, _ = o.ion_flux()
        assert abs(m1 - m0) < 1e-13 * m0
        lows[face] = lo
        if face == 2:
            assert lo >= 0.5 - 1e-13 and hi <= 1.5 + 1e-13
    assert lows[1] < 0.0  # the central form makes the ions negative


def test_z_direction_is_the_x_direction_transposed(oracle_mod):
    ox = _cellular(oracle_mod, 2, "x")
    oz = _cellular(oracle_mod, 2, "z")
    ox.run(60)
    oz.run(60)
    assert abs(ox.t - oz.t) < 1e-13 * ox.t
    cx = ox.field("cp")  # [j][k][i], varies along i
    cz = oz.field("cp")  # varies along k
    np.testing.assert_allclose(cz, np.transpose(cx, (0, 2, 1)), rtol=1e-12, atol=0)
    np.testing.assert_allclose(oz.field("w"), np.transpose(ox.field("u"), (0, 2, 1)), rtol=1e-11, atol=1e-13)


def test_sine_converges_at_second_order(oracle_mod):
    errs = []
    for nx in (32, 64, 128):
        o = _passive(oracle_mod, 2, nx=nx)
        L = nx * o.dx
        k = 2 * np.pi / L
        x = (np.arange(nx) + 0.5) * o.dx
        _set_ions(o, (1 + 0.5 * np.sin(k * x))[None, None, :])
        o.field("u")[...] = 1.0
        while o.t < 2.0 - 1e-12:
            o.run(1)
        D = 1.0 / (o.cfg.re * o.cfg.sc)
        exact = 1 + 0.5 * np.exp(-k * k * D * o.t) * np.sin(k * (x - o.t))
        errs.append(np.mean(np.abs(o.field("cp") - exact[None, None, :])))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.9), (errs, orders)


def test_linear_stretches_match_the_central_form(oracle_mod):
    """A triangle wave in x: cells whose two-cell neighbourhood is linear get
    the central explicit term."""
    nx = 48
    terms = {}
    for face in (1, 2):
        o = _passive(oracle_mod, face, nx=nx)
        i = np.arange(nx)
        tri = 1.0 + np.abs(((i + 0.5) / nx) * 4.0 % 4.0 - 2.0)  # kinks at the faces before cells 0 and 24
        _set_ions(o, tri[None, None, :])
        o.field("u")[...] = np.where(i % 2 == 0, 0.7, -0.4)[None, None, :]
        terms[face] = o.explicit_terms()["cp"][2, 0, :].copy()
    d2 = np.abs(np.roll(tri, -1) - 2 * tri + np.roll(tri, 1)) > 1e-12  # second difference: the kinks
    near = d2 | np.roll(d2, 1) | np.roll(d2, -1)  # cells whose face values see a kink
    assert near.sum() == 8
    np.testing.assert_allclose(terms[2][~near], terms[1][~near], rtol=1e-12, atol=1e-12)
    assert np.max(np.abs(terms[2][near] - terms[1][near])) > 1e-3  # the limiter acts at the kinks


def test_mirrored_profile_and_reversed_flow_mirror_the_result(oracle_mod):
    nx = 32
    rng = np.random.default_rng(3)
    c = 1.0 + 0.5 * rng.uniform(size=nx)
    out = {}
    for sgn in (1.0, -1.0):
        o = _passive(oracle_mod, 2, nx=nx, u_top=sgn, u_bot=sgn)
        _set_ions(o, (c if sgn > 0 else c[::-1])[None, None, :])
        o.field("u")[...] = sgn
        o.run(40)
        out[sgn] = o.field("cp")[2, 0, :].copy()
    np.testing.assert_allclose(out[-1.0], out[1.0][::-1], rtol=1e-13, atol=0)


def test_plane_mean_term_is_minus_the_flux_divergence(oracle_mod):
    """Random velocities of both signs on a stretched grid: the x and z parts
    of the explicit ion term average out over a plane, the wall-normal
    diffusion is implicit, so the plane mean of H is minus the divergence of
    the advective and migration parts of the plane-averaged flux."""
    o = oracle_mod.Oracle(nx=12, ny=15, nz=10, re=300.0, sc=1.0, debye=0.1, vhat=3.0, dt=0.0, cfl=0.5,
                          migration_face=2)
    o.init(4, 0.0, 0.0)
    rng = np.random.default_rng(4)
    sh = o.field("u").shape
    for n in ("u", "v", "w"):
        o.field(n)[...] = rng.standard_normal(sh)
    o.field("v")[0] = 0.0
    o.field("cp")[...] = 1.0 + 0.5 * rng.uniform(size=sh)
    o.field("cm")[...] = 1.0 + 0.5 * rng.uniform(size=sh)
    o.field("phi")[...] = 0.5 * rng.standard_normal(sh)
    h = o.explicit_terms()
    jp, jm, _, _ = o.ion_flux()
    kd = 1.0 / (o.cfg.re * o.cfg.sc)
    M = o.M
    for name, j in (("cp", jp), ("cm", jm)):
        cbar = o.field(name).mean(axis=(1, 2))
        jd = np.zeros(M + 1)
        jd[1:M] = -kd * np.diff(cbar) / o.dc[1:M]
        div = -np.diff(j - jd) / o.dn
        np.testing.assert_allclose(h[name].mean(axis=(1, 2)), div, rtol=1e-10, atol=1e-12 * np.abs(div).max())
