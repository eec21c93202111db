"""GPU (HIP, gfx950) path against the FP64 CPU oracle on the same seeded
inputs, through the C ABI.  Parity measure per field: max|gpu - oracle| /
max|oracle|; the FP64 bar is 1e-10 after the full run."""
import dataclasses
import sys

import numpy as np
import pytest

from inputs import parity, random_field

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


def make_pair(P, O, cfg):
    note(f"case: nx={cfg.nx} ny={cfg.ny} nz={cfg.nz} prec={cfg.precision} dt={cfg.dt} seed={cfg.seed}")
    g = P.Solver(cfg)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    return g, o


def gpu_fields(g):
    g.sync()
    return {k: g.get_field(k).cpu().numpy() for k in FIELDS}


def worst(g, o):
    gf = gpu_fields(g)
    return {k: parity(gf[k], o.field(k)) for k in FIELDS}


SMALL = dict(nx=32, ny=33, nz=32)
RAGGED = dict(nx=48, ny=27, nz=36)       # 2^a 3^b sizes that leave partial tiles everywhere
TINY = dict(nx=6, ny=7, nz=4)


def cfg_of(P, **kw):
    return dataclasses.replace(P.configs.couette_small(), **kw)


@pytest.mark.parametrize("dims", [SMALL, RAGGED, TINY], ids=["small", "ragged", "tiny"])
def test_initial_state_matches_oracle(P, O, dims):
    g, o = make_pair(P, O, cfg_of(P, **dims, seed=3))
    err = worst(g, o)
    assert max(err.values()) < 1e-12, err


@pytest.mark.parametrize("dims", [SMALL, RAGGED], ids=["small", "ragged"])
def test_explicit_terms_match_oracle(P, O, dims):
    g, o = make_pair(P, O, cfg_of(P, **dims, seed=4, u_noise=0.2, c_noise=0.05))
    h = {k: v.cpu().numpy() for k, v in g.explicit_terms().items()}
    ho = o.explicit_terms()
    err = {k: parity(h[k], ho[k]) for k in h}
    assert max(err.values()) < 1e-12, err


# lines of 512 points and more take radix-8 passes: 768 = 8 8 4 3, 512 = 8 8 8
LONG_X = dict(nx=768, ny=9, nz=512)
LONG_Z = dict(nx=512, ny=9, nz=768)


@pytest.mark.parametrize("dims", [SMALL, RAGGED, TINY, LONG_X, LONG_Z], ids=["small", "ragged", "tiny", "long-x", "long-z"])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("thomas", [16, 0], ids=["mode-tiles", "fused-march"])
def test_poisson_solve_matches_oracle(P, O, dims, kind, thomas):
    """Both methods of the y solve: tiles of modes after separate z
    transforms, and the z transforms fused with the y solve into two row
    marches (launch shape thomas = 0)."""
    import torch
    g, o = make_pair(P, O, cfg_of(P, **dims))
    g.set_tiles(thomas=thomas)
    rhs = random_field(o.shape, 10 + kind)
    if kind == 0:
        vol = o.dn[:, None, None] * np.ones(o.shape)
        rhs -= np.sum(rhs * vol) / np.sum(vol)
    t = torch.tensor(rhs, dtype=torch.float64, device="cuda")
    out = g.poisson_solve(kind, t).cpu().numpy()
    ref = o.poisson(kind, rhs)
    # two FFT implementations of different rounding order: their difference
    # grows with the plane size (393 216 points on the long grids, where the
    # zero-flux pressure operator's low modes amplify it to ~1.6e-12); the
    # bar stays well below the 1e-10 of whole-step parity
    bar = 1e-11 if dims in (LONG_X, LONG_Z) else 1e-12
    assert parity(out, ref) < bar


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("cnslab", [0, 16])
def test_small_case_200_substeps_match_oracle(P, O, cnslab, seed):
    """32x33x32, Re 400, lam 0.1, vhat 5, dt 1e-3: 200 RK substeps, with the
    lane-scan (0) and the row-slab (16 rows) Crank-Nicolson methods, for
    seeds 0, 1 and 2."""
    g, o = make_pair(P, O, P.configs.couette_small(seed=seed))
    g.set_tiles(cnslab=cnslab)
    assert g.tiles()["cnslab"] == cnslab
    for chunk in range(4):
        g.step(50)
        o.run(50)
        err = worst(g, o)
        note(f"after {50 * (chunk + 1)} substeps: {max(err.values()):.3e}")
        assert max(err.values()) < 1e-10, err
    tb, tt = g.wall_shear_stress()
    otb, ott = o.wall_shear()
    assert abs(tb - otb) < 1e-10 * abs(otb) and abs(tt - ott) < 1e-10 * abs(ott)
    jp, jm, mp, mm = g.ion_flux()
    ojp, ojm, omp, omm = o.ion_flux()
    assert jp[0] == 0.0 and jp[-1] == 0.0 and jm[0] == 0.0 and jm[-1] == 0.0
    scale = max(np.max(np.abs(ojp)), 1e-30)
    assert np.max(np.abs(np.array(jp) - ojp)) < 1e-10 * scale
    assert abs(mp - omp) < 1e-12 * omp and abs(mm - omm) < 1e-12 * omm
    t, dt, stage, ns = g.clock()
    assert ns == 200 and stage == 200 % 3
    assert abs(t - o.t) < 1e-14
    d = g.diagnostics()
    assert d["max_div"] < 1e-12
    assert abs(d["ke"] - o.kinetic_energy()) < 1e-12 * o.kinetic_energy()


def test_small_case_fused_elliptic_march_matches_oracle(P, O):
    """The 200-substep small case with the z transforms and y solves fused
    into row marches (thomas = 0), both operators every substep."""
    g, o = make_pair(P, O, P.configs.couette_small(seed=1))
    g.set_tiles(thomas=0)
    g.step(200)
    o.run(200)
    err = worst(g, o)
    note(f"fused elliptic march, 200 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err


def test_ragged_adaptive_case_matches_oracle(P, O):
    """48x27x36 with the adaptive time step: 30 substeps."""
    cfg = cfg_of(P, **RAGGED, dt=0.0, cfl=0.5, re=800.0, vhat=8.0, debye=0.08, seed=5, u_noise=0.05)
    g, o = make_pair(P, O, cfg)
    g.step(30)
    o.run(30)
    err = worst(g, o)
    assert max(err.values()) < 1e-10, err
    t, dt, _, _ = g.clock()
    assert abs(dt - o.dt) < 1e-13 * o.dt and abs(t - o.t) < 1e-13


def test_printed_force_sign_matches_oracle(P, O):
    cfg = cfg_of(P, nx=16, ny=17, nz=12, force_sign=1.0, re=100.0, debye=0.2, vhat=6.0, u_noise=0.05, seed=9)
    g, o = make_pair(P, O, cfg)
    g.step(21)
    o.run(21)
    err = worst(g, o)
    assert max(err.values()) < 1e-10, err


# Mixed-form bars per field (max |gpu - oracle| / max |oracle|).  The FP32
# state is rounded every substep, 2^-24 of each value: over n substeps the
# O(1) fields u, c+, c- drift by about n 2^-24 (~4e-6 at n = 60): bar 1e-5.
# v and w are perturbations about 1e-2 of the shear flow, so the same
# absolute rounding is up to ~1e2 times larger relative to their own scale:
# bar 1e-4.  p is the smallest field (pressure increments of the projection):
# bar 1e-2.  phi is solved from the charge c+ - c-, a small difference of two
# O(1) concentrations: through the same linear solve its relative error is at
# most the charge's, i.e. about 2 * 1e-5 * max(c) / max|c+ - c-|, taken with
# a factor 2.
MIXED_BARS = {"u": 1e-5, "v": 1e-4, "w": 1e-4, "cp": 1e-5, "cm": 1e-5, "p": 1e-2}


def mixed_bars(o):
    c = max(np.max(np.abs(o.field("cp"))), np.max(np.abs(o.field("cm"))))
    rho = np.max(np.abs(o.field("cp") - o.field("cm")))
    return {**MIXED_BARS, "phi": 4e-5 * c / rho}


def test_mixed_precision_tracks_oracle(P, O):
    """FP32 state and stencils, FP64 solves: errors at FP32 rounding level,
    every field within its bar."""
    g, o = make_pair(P, O, P.configs.couette_small(precision="mixed", seed=0))
    g.step(60)
    o.run(60)
    err = worst(g, o)
    bars = mixed_bars(o)
    note(f"mixed errors: {err}; bars {bars}")
    for k, bar in bars.items():
        assert err[k] < bar, (k, err)
    tb, tt = g.wall_shear_stress()
    otb, ott = o.wall_shear()
    assert abs(tb - otb) < 1e-4 * otb and abs(tt - ott) < 1e-4 * ott


@pytest.fixture(scope="module")
def turbulent_oracle(P, O):
    """The oracle's 256x193x256 run (Re 3000, lam 0.05, vhat 10, adaptive
    dt): initial state and the state after 30 substeps (ten RK steps)."""
    O.set_threads(16)
    cfg = P.configs.couette_turbulent(seed=0)
    note("oracle: 256x193x256, initial state and 30 substeps")
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    init = o.state()
    o.run(30)
    return dict(init=init, final=o.state(), dt=o.dt, t=o.t, tau=o.wall_shear())


@pytest.mark.parametrize("cnslab,cn,thomas", [(0, 256, 16), (0, 512, 16), (16, 256, 16), (32, 256, 16), (32, 256, 0)])
def test_full_size_turbulent_case_matches_oracle(P, turbulent_oracle, cnslab, cn, thomas):
    """256x193x256, Re 3000, lam 0.05, vhat 10, adaptive dt: initial state
    and 30 substeps (ten RK steps), with each Crank-Nicolson method the
    autotuner can pick (the other launch shapes do not change the arithmetic
    done per cell, line or mode)."""
    ref = turbulent_oracle
    cfg = P.configs.couette_turbulent(seed=0)
    note(f"case: 256x193x256 fp64 cnslab={cnslab} cn={cn} thomas={thomas}, 30 substeps")
    g = P.Solver(cfg)
    g.set_tiles(cnslab=cnslab, cn=cn, thomas=thomas)
    gf = gpu_fields(g)
    err0 = {k: parity(gf[k], ref["init"][k]) for k in FIELDS}
    note(f"full size, initial state: {max(err0.values()):.3e}")
    assert max(err0.values()) < 1e-12, err0
    g.step(30)
    gf = gpu_fields(g)
    err = {k: parity(gf[k], ref["final"][k]) for k in FIELDS}
    note(f"full size, 30 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err
    t, dt, _, _ = g.clock()
    assert abs(dt - ref["dt"]) < 1e-13 * ref["dt"] and abs(t - ref["t"]) < 1e-13 * ref["t"]
    tb, tt = g.wall_shear_stress()
    otb, ott = ref["tau"]
    assert abs(tb - otb) < 1e-10 * otb and abs(tt - ott) < 1e-10 * ott


@pytest.mark.parametrize("dims,cn", [((1024, 513, 4), 256), ((4, 513, 1024), 512), ((1024, 513, 4), 512)],
                         ids=["nx1024-cn16", "nz1024-cn32", "nx1024-cn32"])
def test_maximum_sizes_match_oracle(P, O, dims, cn):
    """The largest supported line lengths (1024 points in x or z) with the
    largest wall-normal count (513 nodes: 512 cell rows, 8 rows per lane in
    the Crank-Nicolson and mode scans, Crank-Nicolson tiles above 64 KB of
    LDS): initial state, then two RK steps with the adaptive time step."""
    nx, ny, nz = dims
    O.set_threads(16)
    cfg = cfg_of(P, nx=nx, ny=ny, nz=nz, dt=0.0, cfl=0.5, re=2000.0, vhat=6.0, debye=0.05, stretch=1.5,
                 seed=3, u_noise=0.05)
    g, o = make_pair(P, O, cfg)
    g.set_tiles(cn=cn)
    err0 = worst(g, o)
    note(f"max size {dims} cn={cn}, initial state: {max(err0.values()):.3e}")
    assert max(err0.values()) < 1e-12, err0
    g.step(6)
    o.run(6)
    err = worst(g, o)
    note(f"max size {dims} cn={cn}, 6 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err
    t, dt, _, _ = g.clock()
    assert abs(dt - o.dt) < 1e-13 * o.dt


def test_maximum_rows_mixed_tracks_oracle(P, O):
    """Mixed form at 513 wall-normal nodes (FP32 state through 32-column
    Crank-Nicolson tiles of 512 rows)."""
    O.set_threads(16)
    cfg = cfg_of(P, nx=64, ny=513, nz=16, precision="mixed", re=2000.0, vhat=6.0, debye=0.05, stretch=1.5,
                 seed=4, u_noise=0.05)
    g, o = make_pair(P, O, cfg)
    g.step(9)
    o.run(9)
    err = worst(g, o)
    bars = mixed_bars(o)
    note(f"mixed, 513 nodes: {err}; bars {bars}")
    for k, bar in bars.items():
        assert err[k] < bar, (k, err)
