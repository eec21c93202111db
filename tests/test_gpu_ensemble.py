"""Ensemble path (all members of a size class in one launch per kernel,
hipGraph replay, autotuned launch shapes) against standalone single runs of
the same configurations, which the parity tests tie to the oracle."""
import dataclasses
import sys

import numpy as np
import pytest

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


def mini_members(P, precision="fp64"):
    base = P.configs.couette_small(precision=precision)
    a = dict(nx=16, ny=17, nz=12)
    b = dict(nx=12, ny=13, nz=8)
    return [
        dataclasses.replace(base, **a, re=300.0, vhat=4.0, debye=0.15, dt=0.0, seed=11, u_noise=0.05),
        dataclasses.replace(base, **b, re=500.0, vhat=8.0, debye=0.2, dt=0.0, seed=12, u_noise=0.05),
        dataclasses.replace(base, **a, re=900.0, vhat=0.0, debye=0.08, dt=0.0, seed=13, u_noise=0.05),
        dataclasses.replace(base, **b, re=200.0, vhat=12.0, debye=0.12, dt=0.0, seed=14, u_noise=0.05),
    ]


def fields_member(e, m):
    return {k: e.get_field(m, k).cpu().numpy() for k in FIELDS}


def test_members_equal_standalone_runs(P):
    cfgs = mini_members(P)
    note("case: 4-member ensemble (2 size classes), 30 substeps vs standalone runs")
    e = P.Ensemble(cfgs)
    assert e.classes() == 2
    e.step(30)
    e.sync()
    for m, c in enumerate(cfgs):
        g = P.Solver(c)
        g.step(30)
        g.sync()
        fe = fields_member(e, m)
        for k in FIELDS:
            a = g.get_field(k).cpu().numpy()
            assert np.array_equal(fe[k], a), (m, k, np.max(np.abs(fe[k] - a)))
        t, dt, ns = e.clock(m)
        tg, dtg, _, _ = g.clock()
        assert ns == 30 and t == tg and dt == dtg
        assert e.wall_shear_stress(m) == g.wall_shear_stress()


def test_graph_replays_match_eager_steps(P):
    cfgs = mini_members(P)
    note("case: 4-member ensemble, graph of 6 substeps replayed 4 times vs eager")
    eg = P.Ensemble(cfgs)
    ee = P.Ensemble(cfgs)
    eg.capture(6)
    for rep in range(4):
        eg.step(6)
        ee.step(6)
        # eager work of the program between replays
        fg = fields_member(eg, rep % len(cfgs))
        fe = fields_member(ee, rep % len(cfgs))
        for k in FIELDS:
            assert np.array_equal(fg[k], fe[k]), (rep, k)
    for m in range(len(cfgs)):
        assert eg.clock(m) == ee.clock(m)


def test_autotuned_shapes_do_not_change_results(P, tmp_path):
    cfgs = mini_members(P, precision="mixed")
    note("case: 4-member mixed ensemble, autotune vs default launch shapes")
    et = P.Ensemble(cfgs)
    tiles = et.autotune(str(tmp_path / "tiles.txt"), trial_substeps=3)
    assert len(tiles) == 2
    _, _, ns = et.clock(0)
    assert all(et.clock(m)[2] == ns for m in range(len(cfgs)))
    ed = P.Ensemble(cfgs)
    ed.step(ns)
    et.step(6)
    ed.step(6)
    # the shapes change no arithmetic except the rounding order of the CN
    # method, which the trials may switch (FP32 state: a few ulps)
    for m in range(len(cfgs)):
        ft, fd = fields_member(et, m), fields_member(ed, m)
        for k in FIELDS:
            scale = max(np.max(np.abs(fd[k])), 1e-30)
            assert np.max(np.abs(ft[k] - fd[k])) <= 1e-5 * scale, (m, k)
    # second tuning reads the cache and gives the same shapes
    assert et.autotune(str(tmp_path / "tiles.txt"), trial_substeps=3) == tiles


def test_time_mean_profiles_of_a_steady_couette_member(P):
    base = P.configs.couette_small()
    c = dataclasses.replace(base, nx=12, ny=17, nz=8, vhat=0.0, u_noise=0.0, c_noise=0.0, dt=2e-3)
    note("case: steady Couette member, statistics over 9 substeps")
    e = P.Ensemble([c, c])
    e.stats(True)
    e.step(9)
    u, rho, phi, wt = e.profiles(1)
    g = P.Solver(c)
    yc = g.get_field("u").cpu().numpy()[:, 0, 0]
    assert wt == pytest.approx(3 * 2e-3, rel=1e-12)
    assert np.max(np.abs(np.array(u) - yc)) < 1e-13
    assert np.max(np.abs(rho)) < 1e-14 and np.max(np.abs(phi)) < 1e-14


def test_single_run_autotune_does_not_change_results(P):
    cfg = dataclasses.replace(P.configs.couette_small(), nx=48, ny=27, nz=36, dt=0.0, cfl=0.5, seed=5)
    note("case: single-run autotune 48x27x36")
    a = P.Solver(cfg)
    tiles = a.autotune(None, 3)
    note(f"  tiles {tiles}")
    n = a.clock()[3]
    b = P.Solver(cfg)
    b.step(n)
    a.step(6)
    b.step(6)
    # identical arithmetic per cell except the CN rounding order (FP64)
    for k in ("u", "v", "w", "cp", "cm", "phi", "p"):
        fa, fb = a.get_field(k).cpu().numpy(), b.get_field(k).cpu().numpy()
        assert np.max(np.abs(fa - fb)) <= 1e-12 * max(np.max(np.abs(fb)), 1e-30), k


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as mod
    mod._load()
    return mod


# Mixed-form bars per field (max |gpu - oracle| / max |oracle|): the FP32
# state is rounded every substep (2^-24 relative to the field's own scale,
# accumulating over ~150 substeps to ~1e-5 for u and c+-): bar 2e-5; v and w
# are perturbations of the O(1) shear flow, so the same absolute rounding is
# up to ~1e2 larger relative to their scale: 2e-3; p is the smallest field:
# 2e-2; phi follows the charge, a small difference of two O(1)
# concentrations, so its relative error is the charge's: 4 * 2e-5 * max(c) /
# max|c+ - c-|.
MIXED_BARS = {"u": 2e-5, "v": 2e-3, "w": 2e-3, "cp": 2e-5, "cm": 2e-5, "p": 2e-2}


def mixed_bars(o):
    c = max(np.max(np.abs(o.field("cp"))), np.max(np.abs(o.field("cm"))))
    rho = np.max(np.abs(o.field("cp") - o.field("cm")))
    return {**MIXED_BARS, "phi": 8e-5 * c / rho}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_production_size_members_match_oracle(P, O, precision):
    """One member of each size class of the production ensemble (64x65x64
    and 48x49x48, parameters from the ensemble sampler), batched in one
    ensemble with autotuned launch shapes, against the oracle after the
    tuner's trial substeps plus 30 more: FP64 within 1e-10 per field, the
    mixed form within its per-field bars."""
    members = P.configs.ensemble_members(seed=0, precision=precision)
    pick = [members[0], members[32]]
    note(f"case: ensemble members 0 (64x65x64) and 32 (48x49x48), {precision}, autotuned + 30 substeps")
    e = P.Ensemble(pick)
    assert e.classes() == 2
    tiles = e.autotune(None, 3)
    note(f"  tiles {tiles}")
    e.step(30)
    e.sync()
    O.set_threads(16)
    for m, c in enumerate(pick):
        t, dt, ns = e.clock(m)
        o = O.Oracle(**c.oracle_kwargs())
        o.init(c.seed, c.u_noise, c.c_noise)
        o.run(ns)
        fe = fields_member(e, m)
        err = {k: float(np.max(np.abs(fe[k] - o.field(k))) / max(np.max(np.abs(o.field(k))), 1e-300))
               for k in FIELDS}
        note(f"  member {m} ({c.nx}x{c.ny}x{c.nz}, Re {c.re:.0f}, vhat {c.vhat:.2f}, lam {c.debye:.4f}) "
             f"after {ns} substeps: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()))
        if precision == "fp64":
            assert max(err.values()) < 1e-10, err
            assert abs(dt - o.dt) < 1e-13 * o.dt and abs(t - o.t) < 1e-13 * max(o.t, 1.0)
        else:
            bars = mixed_bars(o)
            note(f"  bars {bars}")
            for k, bar in bars.items():
                assert err[k] < bar, (k, err)
            assert abs(dt - o.dt) < 1e-5 * o.dt
