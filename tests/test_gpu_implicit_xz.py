"""Three-direction approximate factorisation of the HIP path (config
implicit_xz = 1: diffusion implicit in x, y and z) against the oracle on the
same seeded runs, through the C ABI.  The periodic x/z line solves (cyclic
tridiagonals by recurrences and a rank-one correction on the GPU, Fourier
division in the oracle) are exercised at every line length class, including
lines that need the large-LDS launch."""
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
    cfg = dataclasses.replace(P.configs.couette_small(), implicit_xz=1, **kw)
    note(f"case: implicit_xz {cfg.nx}x{cfg.ny}x{cfg.nz} {cfg.precision} dt={cfg.dt} re={cfg.re} seed={cfg.seed}")
    g = P.Solver(cfg)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    return cfg, g, o


def worst(g, o):
    g.sync()
    return {k: parity(g.get_field(k).cpu().numpy(), o.field(k)) for k in FIELDS}


def test_small_case_matches_oracle(P, O):
    cfg, g, o = pair(P, O, seed=0)
    g.step(60)
    o.run(60)
    err = worst(g, o)
    note(f"60 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err


def test_ragged_adaptive_case_matches_oracle(P, O):
    cfg, g, o = pair(P, O, nx=48, ny=27, nz=36, dt=0.0, cfl=0.5, re=800.0, vhat=8.0, debye=0.08, seed=5,
                     u_noise=0.05)
    g.step(30)
    o.run(30)
    err = worst(g, o)
    assert max(err.values()) < 1e-10, err
    t, dt, _, _ = g.clock()
    assert abs(dt - o.dt) < 1e-13 * o.dt


def test_beyond_the_explicit_diffusion_limit(P, O):
    """Re 20 on 32x17x32: a fixed dt three times the explicit x/z diffusion
    limit, which the factorisation allows."""
    cfg0 = dataclasses.replace(P.configs.couette_small(), nx=32, ny=17, nz=32, re=20.0)
    dx, dz = cfg0.lx / cfg0.nx, cfg0.lz / cfg0.nz
    limit = cfg0.re / (4 / dx ** 2 + 4 / dz ** 2)
    cfg, g, o = pair(P, O, nx=32, ny=17, nz=32, re=20.0, dt=3 * limit, seed=2, u_noise=0.05)
    g.step(45)
    o.run(45)
    err = worst(g, o)
    assert max(err.values()) < 1e-10, err
    assert g.diagnostics()["max_div"] < 1e-12


@pytest.mark.parametrize("dims", [(512, 9, 8), (8, 9, 1024)], ids=["nx512", "nz1024"])
def test_long_periodic_lines(P, O, dims):
    nx, ny, nz = dims
    cfg, g, o = pair(P, O, nx=nx, ny=ny, nz=nz, seed=3, re=200.0)
    g.step(9)
    o.run(9)
    err = worst(g, o)
    assert max(err.values()) < 1e-10, err


def test_mixed_precision_tracks_oracle(P, O):
    cfg, g, o = pair(P, O, precision="mixed", seed=0)
    g.step(60)
    o.run(60)
    err = worst(g, o)
    note(f"mixed: {err}")
    for k in ("u", "cp", "cm"):
        assert err[k] < 1e-5, err


def test_full_size_case_matches_oracle(P, O):
    O.set_threads(16)
    cfg, g, o = pair(P, O, **{k: v for k, v in dataclasses.asdict(P.configs.couette_turbulent(seed=0)).items()
                             if k in ("nx", "ny", "nz", "re", "debye", "vhat", "dt", "cfl", "seed")})
    g.step(3)
    o.run(3)
    err = worst(g, o)
    note(f"full size, 3 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err


def test_cn_tile_width_is_bitwise_neutral(P):
    import torch
    cfg = dataclasses.replace(P.configs.couette_small(), nx=36, ny=27, nz=18, implicit_xz=1, seed=6,
                              dt=0.0, cfl=0.5)
    a, b = P.Solver(cfg), P.Solver(cfg)
    b.set_tiles(cn=512, expl=128, corr=64)
    a.step(9)
    b.step(9)
    for k in FIELDS:
        assert torch.equal(a.get_field(k).cpu(), b.get_field(k).cpu()), k
