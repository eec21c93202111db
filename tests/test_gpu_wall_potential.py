"""Arbitrary wall potential of the HIP path (nspnp_set_wall_potential)
against the oracle's inhomogeneous Dirichlet potential on the same seeded
runs, through the C ABI: the potential solve alone, coupled substeps with a
fixed wall pattern, and a travelling wall wave updated between steps."""
import dataclasses
import math
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
    cfg = dataclasses.replace(P.configs.couette_small(), **kw)
    note(f"case: wall potential {cfg.nx}x{cfg.ny}x{cfg.nz} vhat={cfg.vhat} seed={cfg.seed}")
    g = P.Solver(cfg)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    return cfg, g, o


def pattern(cfg, t=0.0, amp=1.5, speed=0.0, m=1, n=1):
    """amp cos(a (x - speed t)) cos(b z) at the cell columns ([nz, nx])."""
    x = (np.arange(cfg.nx) + 0.5) * (cfg.lx / cfg.nx)
    z = (np.arange(cfg.nz) + 0.5) * (cfg.lz / cfg.nz)
    a, b = 2 * math.pi * m / cfg.lx, 2 * math.pi * n / cfg.lz
    return amp * np.cos(b * z)[:, None] * np.cos(a * (x - speed * t))[None, :]


def set_both(g, o, bot, top):
    import torch
    tb = None if bot is None else torch.tensor(bot, dtype=torch.float64, device="cuda")
    tt = None if top is None else torch.tensor(top, dtype=torch.float64, device="cuda")
    g.set_wall_potential(tb, tt)
    o.set_wall_potential(bot, top)


def worst(g, o):
    g.sync()
    return {k: parity(g.get_field(k).cpu().numpy(), o.field(k)) for k in FIELDS}


@pytest.mark.parametrize("dims", [(32, 33, 32), (48, 27, 36)], ids=["32x33x32", "48x27x36"])
def test_potential_solve_with_wall_values(P, O, dims):
    nx, ny, nz = dims
    cfg, g, o = pair(P, O, nx=nx, ny=ny, nz=nz, seed=2)
    bot, top = pattern(cfg), -0.5 * pattern(cfg, m=2, n=1)
    set_both(g, o, bot, top)
    g.refresh_potential()
    o.solve_potential()
    g.sync()
    err = parity(g.get_field("phi").cpu().numpy(), o.field("phi"))
    note(f"phi parity {err:.3e}")
    assert err < 1e-12


def test_substeps_with_a_wall_pattern(P, O):
    cfg, g, o = pair(P, O, seed=0, vhat=5.0)
    set_both(g, o, pattern(cfg, amp=1.0), pattern(cfg, amp=0.7, n=2))
    g.refresh_potential()
    o.solve_potential()
    g.step(30)
    o.run(30)
    err = worst(g, o)
    note(f"after 30 substeps: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err


def test_travelling_wall_wave(P, O):
    cfg, g, o = pair(P, O, seed=4, vhat=2.0)
    t = 0.0
    for k in range(4):
        bot = pattern(cfg, t=t, amp=2.0, speed=3.0)
        set_both(g, o, bot, None)
        g.step(6)
        o.run(6)
        t = o.t
    err = worst(g, o)
    note(f"travelling wave: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err


def test_cleared_wall_values_restore_uniform_walls(P):
    import torch
    cfg = dataclasses.replace(P.configs.couette_small(), seed=6)
    a, b = P.Solver(cfg), P.Solver(cfg)
    g0 = torch.tensor(pattern(cfg), dtype=torch.float64, device="cuda")
    b.set_wall_potential(g0, g0)
    b.set_wall_potential(None, None)
    a.step(9)
    b.step(9)
    for k in FIELDS:
        assert torch.equal(a.get_field(k).cpu(), b.get_field(k).cpu()), k
