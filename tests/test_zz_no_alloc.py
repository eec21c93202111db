"""nspnp_poisson_solve_noalloc (the elliptic solve on the library's fixed
device scratch, no handle, no workspace) against nspnp_poisson_solve on a
handle of the same grid, through the C ABI: two calls in a row, the second
on a smaller grid, then the first grid again; both elliptic kinds.  The two
entry points run the same kernels on the same tables and pivots, so they must
agree to the parity bar of the elliptic solve (1e-12 relative)."""
import dataclasses
import sys

import numpy as np
import pytest

from inputs import parity, random_field

pytestmark = pytest.mark.gpu


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


def rhs_for(cfg, kind, seed):
    M = cfg.ny - 1
    r = random_field((M, cfg.nz, cfg.nx), seed)
    if kind == 0:  # the pressure operator needs a zero volume-mean right side
        from paper_1701_02005_amd import grid
        yn, _ = grid(cfg)
        dn = np.diff(np.array(yn))[:, None, None] * np.ones_like(r)
        r -= np.sum(r * dn) / np.sum(dn)
    return r


def solve_both(P, cfg, kind, seed):
    import torch
    rhs = torch.tensor(rhs_for(cfg, kind, seed), dtype=torch.float64, device="cuda")
    out = torch.full_like(rhs, float("nan"))
    P.poisson_solve_noalloc(cfg, kind, rhs, out)
    torch.cuda.synchronize()
    g = P.Solver(cfg)
    ref = g.poisson_solve(kind, rhs)
    g.sync()
    return out.cpu().numpy(), ref.cpu().numpy()


LARGER = dict(nx=48, ny=27, nz=36)    # ragged tiles in every direction
SMALLER = dict(nx=16, ny=17, nz=12)


@pytest.mark.parametrize("kind", [0, 1])
def test_noalloc_matches_handle_solve_twice(P, kind):
    base = P.configs.couette_small()
    for step, dims in enumerate((LARGER, SMALLER, LARGER)):
        cfg = dataclasses.replace(base, **dims)
        note(f"case: poisson_solve_noalloc kind {kind}, call {step + 1}, grid {dims}")
        a, b = solve_both(P, cfg, kind, seed=20 + 3 * step + kind)
        err = parity(a, b)
        note(f"  max |noalloc - handle| / max |handle| = {err:.3e}")
        assert np.all(np.isfinite(a))
        assert err <= 1e-12


def test_noalloc_repeated_calls_on_one_grid(P):
    """Later calls on the same grid reuse the tables and pivots in the
    scratch: a different right-hand side gives its own solution."""
    import torch
    cfg = dataclasses.replace(P.configs.couette_small(), **SMALLER)
    note("case: poisson_solve_noalloc, three right-hand sides on one grid")
    g = P.Solver(cfg)
    for seed in (31, 32, 33):
        rhs = torch.tensor(rhs_for(cfg, 1, seed), dtype=torch.float64, device="cuda")
        a = P.poisson_solve_noalloc(cfg, 1, rhs)
        b = g.poisson_solve(1, rhs)
        torch.cuda.synchronize()
        assert parity(a.cpu().numpy(), b.cpu().numpy()) <= 1e-12


def test_noalloc_refuses_grids_beyond_its_scratch(P):
    import torch
    cfg = P.configs.couette_turbulent()  # 256x193x256: ~300 MB of spectrum and pivots
    note("case: poisson_solve_noalloc refuses 256x193x256")
    x = torch.zeros(cfg.cells, dtype=torch.float64, device="cuda")
    with pytest.raises(P.NsPnpError) as e:
        P.poisson_solve_noalloc(cfg, 0, x, x)
    assert e.value.code == -2 and "scratch" in str(e.value)
    small = dataclasses.replace(P.configs.couette_small(), **SMALLER)
    y = torch.zeros(small.cells, dtype=torch.float64, device="cuda")
    with pytest.raises(P.NsPnpError) as e:
        P.poisson_solve_noalloc(small, 2, y, y)
    assert e.value.code == -1
