"""Run statistics of the HIP path (nspnp_stats_begin / nspnp_stats_read)
against the oracle's written-out definition (oracle/stats_oracle.py) on the
same seeded runs, through the C ABI: time-weighted plane means and mean
squares of the seven fields, the wall quantities derived from them, and
their continuation across a checkpoint."""
import dataclasses
import math
import sys

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as mod
    mod._load()
    return mod


@pytest.fixture(scope="module")
def S():
    from oracle import stats_oracle as mod
    return mod


def cfg_of(P, **kw):
    return dataclasses.replace(P.configs.couette_small(), **kw)


def run_pair(P, O, S, cfg, nsub, every):
    """GPU run with sampling every `every` substeps, and the oracle sampled at
    the same substeps with the reference definition."""
    note(f"case: stats {cfg.nx}x{cfg.ny}x{cfg.nz} {cfg.precision} dt={cfg.dt} every={every} nsub={nsub}")
    g = P.Solver(cfg)
    g.stats_begin(every)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    ta = S.TimeAverage(o.t)
    for n in range(1, nsub + 1):
        o.substep()
        if n % every == 0:
            ta.sample(o.t, o.state())
    g.step(nsub)
    T, ns, st = g.stats_read()
    return g, o, ta, T, ns, st


def rel_err(st, ref, names):
    """Error of each time average relative to its scale: the largest |value|
    for mean squares, and for means the larger of the largest |mean| and the
    field's RMS size sqrt(max <q^2>) (the plane mean of v vanishes by
    continuity, so only rounding noise is left to divide by)."""
    nf = len(names) // 2
    out = {}
    for q, k in enumerate(names):
        a, b = np.asarray(st[k]), ref[q]
        scale = np.max(np.abs(b))
        if q < nf:
            scale = max(scale, math.sqrt(np.max(ref[q + nf])))
        out[k] = float(np.max(np.abs(a - b)) / max(scale, 1e-300))
    return out


@pytest.mark.parametrize("case", ["fixed_every1", "adaptive_every3_ragged"])
def test_statistics_match_oracle(P, O, S, case):
    if case == "fixed_every1":
        cfg, nsub, every = cfg_of(P, seed=0), 30, 1
    else:
        cfg = cfg_of(P, nx=48, ny=27, nz=36, dt=0.0, cfl=0.5, re=800.0, vhat=8.0, debye=0.08, seed=5, u_noise=0.05)
        nsub, every = 30, 3
    g, o, ta, T, ns, st = run_pair(P, O, S, cfg, nsub, every)
    assert ns == ta.samples == nsub // every
    assert abs(T - ta.time) < 1e-13 * ta.time
    err = rel_err(st, ta.averages(), P.binding.STATS_NAMES)
    note(f"stats parity: {max(err.values()):.3e}")
    assert max(err.values()) < 1e-10, err
    # derived wall quantities against the reference formulas
    d = g.statistics()
    wq = S.wall_quantities(ta.averages()[0], o.yn, cfg.re, cfg.u_bot, cfg.u_top)
    for k in ("tau_bottom", "tau_top", "cf", "re_tau"):
        assert abs(d[k] - wq[k]) < 1e-10 * abs(wq[k]), k
    ref_rms = S.rms(ta.averages()[3], ta.averages()[10])
    assert np.max(np.abs(np.array(d["rms"]["cp"]) - ref_rms)) < 1e-8 * max(np.max(ref_rms), 1e-30)


def test_mixed_precision_statistics_track_oracle(P, O, S):
    cfg = cfg_of(P, precision="mixed", seed=0)
    g, o, ta, T, ns, st = run_pair(P, O, S, cfg, 30, 2)
    err = rel_err(st, ta.averages(), P.binding.STATS_NAMES)
    note(f"mixed stats errors: {err}")
    for k in ("u", "u2", "cp", "cm", "cp2", "cm2"):
        assert err[k] < 1e-5, err


def test_laminar_couette_law_of_the_wall(P):
    """No noise and no voltage: exact Couette flow, so the averaged profile is
    linear, u+ = y+ and c_f = 2/Re to rounding."""
    cfg = cfg_of(P, u_noise=0.0, c_noise=0.0, vhat=0.0, seed=1)
    note("case: laminar statistics")
    g = P.Solver(cfg)
    g.stats_begin(1)
    g.step(12)
    d = g.statistics()
    assert d["samples"] == 12
    assert abs(d["cf"] - 2.0 / cfg.re) < 1e-11
    assert abs(d["re_tau"] - math.sqrt(cfg.re)) < 1e-8
    assert np.allclose(d["u_plus"], d["y_plus"], rtol=1e-10)
    assert max(d["rms"]["u"]) < 1e-6


def test_statistics_continue_across_checkpoint(P, tmp_path):
    cfg = cfg_of(P, dt=0.0, cfl=0.5, seed=3)
    note("case: statistics across a checkpoint")
    a = P.Solver(cfg)
    a.stats_begin(2)
    a.step(7)
    path = tmp_path / "stats.ckpt"
    a.save(path)
    a.step(8)
    ref = a.stats_read()
    b = P.Solver(dataclasses.replace(cfg, seed=cfg.seed + 1))
    b.load(path)
    b.step(8)
    got = b.stats_read()
    assert got[0] == ref[0] and got[1] == ref[1] == 7
    for k in P.binding.STATS_NAMES:
        assert got[2][k] == ref[2][k], k
    # stop keeps the sums; begin clears them
    b.stats_begin(0)
    b.step(4)
    assert b.stats_read()[1] == 7
    b.stats_begin(1)
    assert b.stats_read()[1] == 0
