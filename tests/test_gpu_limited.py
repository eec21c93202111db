"""Limited advective face values of the ions (migration_face = 2) on the GPU
against the oracle, which the CPU tests pin (bounds kept by a square wave and
a stirred blob, second-order convergence, mirror symmetry, the central form
on linear stretches, flux consistency).  Velocities of both signs reach every
branch of the upwind choice; wall rows are in every case."""
import dataclasses
import sys

import numpy as np
import pytest

from inputs import parity

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "w", "cp", "cm", "phi", "p")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02005_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as mod
    mod._load()
    return mod


def pair(P, O, **kw):
    cfg = dataclasses.replace(P.configs.couette_small(), migration_face=2, **kw)
    note(f"case: limited advection {cfg.nx}x{cfg.ny}x{cfg.nz} re={cfg.re} vhat={cfg.vhat} lam={cfg.debye} "
         f"{cfg.precision} seed={cfg.seed}")
    g = P.Solver(cfg)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    return cfg, g, o


def put(g, o, name, val):
    import torch
    o.field(name)[...] = val
    g.set_field(name, torch.tensor(np.ascontiguousarray(o.field(name)), dtype=torch.float64, device="cuda"))


def errors(g, o):
    g.sync()
    return {k: parity(g.get_field(k).cpu().numpy(), o.field(k)) for k in FIELDS}


SMALL = dict(nx=16, ny=9, nz=8, re=800.0, debye=0.08, vhat=8.0, dt=0.0, cfl=0.5, seed=5, u_noise=0.3)
RAGGED = dict(nx=48, ny=13, nz=36, re=2000.0, debye=0.05, vhat=20.0, dt=0.0, cfl=0.5, seed=6, u_noise=0.3)


@pytest.mark.parametrize("dims", [SMALL, RAGGED], ids=["small", "ragged"])
def test_explicit_terms_with_random_velocities(P, O, dims):
    cfg, g, o = pair(P, O, **dims)
    rng = np.random.default_rng(7)
    sh = o.shape
    for k in ("u", "v", "w"):
        val = rng.standard_normal(sh)
        if k == "v":
            val[0] = 0.0
        put(g, o, k, val)
    for k in ("cp", "cm"):
        put(g, o, k, 1.0 + 0.8 * rng.uniform(size=sh))
    put(g, o, "phi", rng.standard_normal(sh))
    h = {k: v.cpu().numpy() for k, v in g.explicit_terms().items()}
    ho = o.explicit_terms()
    err = {k: parity(h[k], ho[k]) for k in h}
    note(f"  explicit terms: {err}")
    assert max(err.values()) < 1e-12, err


@pytest.mark.parametrize("dims", [SMALL, RAGGED], ids=["small", "ragged"])
def test_limited_run_matches_oracle(P, O, dims):
    cfg, g, o = pair(P, O, **dims)
    for chunk in range(3):
        g.step(20)
        o.run(20)
        err = errors(g, o)
        note(f"  after {20 * (chunk + 1)} substeps: {max(err.values()):.3e}")
        assert max(err.values()) < 1e-10, err
    t, dt, _, _ = g.clock()
    assert abs(dt - o.dt) < 1e-13 * o.dt and abs(t - o.t) < 1e-13 * o.t
    jp, jm, mp, mm = g.ion_flux()
    ojp, ojm, omp, omm = o.ion_flux()
    scale = max(np.max(np.abs(ojp)), np.max(np.abs(ojm)))
    assert np.max(np.abs(np.array(jp) - ojp)) < 1e-10 * scale
    assert np.max(np.abs(np.array(jm) - ojm)) < 1e-10 * scale
    assert abs(mp - omp) < 1e-12 * omp and abs(mm - omm) < 1e-12 * omm


@pytest.mark.parametrize("cnslab", [0, 16, 32])
def test_limited_run_with_each_cn_method(P, O, cnslab):
    """The limited correction after the explicit kernel under the lane-scan
    (0) and the row-slab (16, 32 rows) Crank-Nicolson methods: the row-slab
    method's first pass ran inside the explicit kernel on the uncorrected r,
    and the correction pass adds the slab exits of its own change of r."""
    cfg, g, o = pair(P, O, nx=32, ny=65, nz=24, re=1500.0, debye=0.06, vhat=12.0, dt=0.0, cfl=0.5, seed=9,
                     u_noise=0.3)
    g.set_tiles(cnslab=cnslab)
    assert g.tiles()["cnslab"] == cnslab
    for chunk in range(3):
        g.step(20)
        o.run(20)
        err = errors(g, o)
        note(f"  cnslab {cnslab}, after {20 * (chunk + 1)} substeps: {max(err.values()):.3e}")
        assert max(err.values()) < 1e-10, err


def test_stirred_blob_keeps_bounds_on_the_gpu(P, O):
    """Uncharged ions (vhat 0, c+ = c-) in a discretely divergence-free
    cellular flow between the walls: the limited update keeps the blob
    within its initial bounds, and the state follows the oracle's."""
    cfg, g, o = pair(P, O, nx=32, ny=33, nz=4, re=1e3, sc=10.0, vhat=0.0, beta=0.0, u_top=0.0, u_bot=0.0,
                     debye=0.1, dt=0.0, cfl=0.5, seed=0, u_noise=0.0, c_noise=0.0)
    M, nx = o.M, cfg.nx
    L = nx * o.dx
    xf = np.arange(nx) * o.dx
    psi = np.sin(2 * np.pi * xf / L)[None, :] * np.sin(np.pi * (o.yn[:, None] + 1) / 2)
    u = (psi[1:] - psi[:-1]) / o.dn[:, None]
    v = -(np.roll(psi, -1, axis=1) - psi) / o.dx
    xc = (np.arange(nx) + 0.5) * o.dx
    c = np.where((np.abs(xc - L / 2)[None, :] < L / 4) & (np.abs(o.yc)[:, None] < 0.4), 1.5, 0.5)
    sh = o.shape
    put(g, o, "u", np.broadcast_to(u[:, None, :], sh))
    put(g, o, "v", np.broadcast_to(v[:M][:, None, :], sh))
    for k in ("w", "phi", "p"):
        put(g, o, k, np.zeros(sh))
    for k in ("cp", "cm"):
        put(g, o, k, np.broadcast_to(c[:, None, :], sh))
    lo, hi = np.inf, -np.inf
    while o.t < 3.0:
        g.step(10)
        o.run(10)
        d = g.diagnostics()
        lo = min(lo, d["min_cp"])
        cg = g.get_field("cp").cpu().numpy()
        hi = max(hi, cg.max())
    note(f"  blob bounds on the GPU: [{lo:.17g}, {hi:.17g}]")
    assert lo >= 0.5 - 1e-13 and hi <= 1.5 + 1e-13
    err = errors(g, o)
    # w stays zero up to rounding in this x-y flow: measured against the velocity scale
    w_abs = np.max(np.abs(g.get_field("w").cpu().numpy() - o.field("w")))
    err["w"] = w_abs / np.max(np.abs(o.field("u")))
    assert max(err.values()) < 1e-10, err


def test_limited_mixed_form_tracks_oracle(P, O):
    cfg, g, o = pair(P, O, precision="mixed", **SMALL)
    g.step(60)
    o.run(60)
    err = errors(g, o)
    note(f"  mixed limited: {err}")
    for k in ("u", "cp", "cm"):
        assert err[k] < 1e-5, (k, err)


def test_ensemble_members_with_limited_advection(P):
    """The ensemble path (one launch per kernel for all members) runs the
    limited correction per member: members equal standalone runs."""
    base = dataclasses.replace(P.configs.couette_small(), nx=16, ny=17, nz=12, migration_face=2, dt=0.0,
                               u_noise=0.3)
    cfgs = [dataclasses.replace(base, re=800.0, vhat=4.0, debye=0.1, seed=21),
            dataclasses.replace(base, re=1500.0, vhat=12.0, debye=0.06, seed=22)]
    e = P.Ensemble(cfgs)
    e.step(30)
    e.sync()
    for m, c in enumerate(cfgs):
        g = P.Solver(c)
        g.step(30)
        g.sync()
        for k in FIELDS:
            a = g.get_field(k).cpu().numpy()
            b = e.get_field(m, k).cpu().numpy()
            assert np.array_equal(a, b), (m, k, np.max(np.abs(a - b)))
