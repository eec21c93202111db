"""Health checks, the migration cell-Peclet diagnostic and checkpoints of the
HIP path, through the C ABI.  The faults here are planted in the field
values (NaN, a negative concentration): every kernel still runs its normal,
bounded index range."""
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


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as mod
    mod._load()
    return mod


def small(P, **kw):
    base = dict(nx=16, ny=17, nz=12, re=400.0, debye=0.1, vhat=5.0, dt=1e-3, seed=3)
    base.update(kw)
    return dataclasses.replace(P.configs.couette_small(), **base)


def max_dphi(phi, yc, e0):
    """Largest |Phi difference| across interior faces, Phi = phi + e0 y."""
    tot = phi + e0 * np.asarray(yc)[:, None, None]
    dx = np.abs(np.roll(tot, -1, axis=2) - tot).max()
    dz = np.abs(np.roll(tot, -1, axis=1) - tot).max()
    dy = np.abs(np.diff(tot, axis=0)).max()
    return max(dx, dz, dy)


def test_max_dphi_diagnostic_matches_oracle_fields(P, O):
    cfg = small(P)
    note(f"case: max_dphi {cfg.nx}x{cfg.ny}x{cfg.nz}")
    g = P.Solver(cfg)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    g.step(30)
    o.run(30)
    d = g.diagnostics()
    _, yc = P.grid(cfg)
    ref = max_dphi(o.field("phi"), yc, 0.5 * cfg.vhat)
    assert abs(d["max_dphi"] - ref) <= 1e-10 * ref
    # the same quantity from the GPU's own fields
    assert abs(d["max_dphi"] - max_dphi(g.get_field("phi").cpu().numpy(), yc, 0.5 * cfg.vhat)) <= 1e-12 * ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nonfinite_value_is_reported_and_sticky(P, precision):
    import torch
    cfg = small(P, precision=precision)
    note(f"case: NaN planted, {precision}")
    g = P.Solver(cfg)
    g.step(3)
    g.sync()
    u = g.get_field("u")
    bad = u.clone()
    bad.view(-1)[1234] = float("nan")
    g.set_field("u", bad)
    g.step(1)  # substep 3: stage 0 runs the check
    with pytest.raises(P.NsPnpError) as ei:
        g.sync()
    assert ei.value.code == -4 and "non-finite" in str(ei.value)
    with pytest.raises(P.NsPnpError):
        g.step(1)
    # reset: a new clock clears the flag, then clean fields
    g.set_clock(0.0, cfg.dt, 0, 0)
    g2 = P.Solver(cfg)
    for k in FIELDS:
        g.set_field(k, g2.get_field(k))
    g.step(6)
    g.sync()
    torch.cuda.synchronize()


def test_negative_concentration_is_reported(P):
    cfg = small(P)
    note("case: negative c- planted")
    g = P.Solver(cfg)
    cm = g.get_field("cm")
    cm.view(-1)[77] = -0.5
    g.set_field("cm", cm)
    g.step(1)
    with pytest.raises(P.NsPnpError) as ei:
        g.sync()
    assert ei.value.code == -4 and "negative concentration" in str(ei.value)


def test_healthy_run_passes_the_checks(P):
    cfg = small(P, dt=0.0, cfl=0.5)
    note("case: healthy adaptive run")
    g = P.Solver(cfg)
    for _ in range(4):
        g.step(7)
    g.sync()
    assert g.diagnostics()["min_cp"] > 0.0


def test_ensemble_member_fault_names_the_member(P):
    base = small(P)
    cfgs = [dataclasses.replace(base, seed=s) for s in range(3)] + [
        dataclasses.replace(base, nx=12, nz=8, ny=13, seed=9)]
    note("case: ensemble fault in member 3")
    e = P.Ensemble(cfgs)
    e.step(3)
    e.sync()
    cp = e.get_field(3, "cp")
    cp.view(-1)[5] = -1.0
    e.set_field(3, "cp", cp)
    e.step(3)
    with pytest.raises(P.NsPnpError) as ei:
        e.sync()
    assert "member 3" in str(ei.value)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_restart_is_bitwise(P, precision, tmp_path):
    import torch
    cfg = small(P, precision=precision, dt=0.0, cfl=0.5)
    note(f"case: checkpoint {precision}")
    a = P.Solver(cfg)
    a.step(5)  # stops inside a Runge-Kutta step: H of stage 1 is live
    path = tmp_path / "run.ckpt"
    a.save(path)
    a.step(7)
    ref = {k: a.get_field(k).cpu() for k in FIELDS}
    tref = a.clock()
    b = P.Solver(dataclasses.replace(cfg, seed=cfg.seed + 1))  # other initial noise
    b.load(path)
    assert b.clock()[3] == 5
    b.step(7)
    for k in FIELDS:
        assert torch.equal(b.get_field(k).cpu(), ref[k]), k
    assert b.clock() == tref


def test_checkpoint_rejects_other_configuration(P, tmp_path):
    cfg = small(P)
    note("case: checkpoint mismatch")
    a = P.Solver(cfg)
    path = tmp_path / "run.ckpt"
    a.save(path)
    b = P.Solver(dataclasses.replace(cfg, re=500.0))
    with pytest.raises(P.NsPnpError) as ei:
        b.load(path)
    assert ei.value.code == -1
    junk = tmp_path / "junk"
    junk.write_bytes(b"not a checkpoint")
    with pytest.raises(P.NsPnpError):
        a.load(junk)


def test_set_tiles_validates(P):
    g = P.Solver(small(P))
    t = g.tiles()
    assert t["cnslab"] in (0, 16, 32)
    with pytest.raises(P.NsPnpError):
        g.set_tiles(cnslab=8)
    with pytest.raises(P.NsPnpError):
        g.set_tiles(expl=100)
    g.set_tiles(cnslab=16, thomas=4)
    assert g.tiles()["cnslab"] == 16 and g.tiles()["thomas"] == 4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dims", [(48, 27, 36), (36, 27, 18)], ids=["48x27x36", "36x27x18"])
def test_launch_order_shapes_are_bitwise_neutral(P, precision, dims):
    """Block order and tile shapes that do not change the per-cell, per-line or
    per-mode arithmetic give bitwise identical runs (36x18 columns leave a
    ragged last tile of the 32-column Crank-Nicolson blocks)."""
    import torch
    nx, ny, nz = dims
    cfg = small(P, nx=nx, ny=ny, nz=nz, dt=0.0, cfl=0.5, seed=8, precision=precision)
    note(f"case: launch shapes vs defaults, {nx}x{ny}x{nz} {precision}")
    a = P.Solver(cfg)
    b = P.Solver(cfg)
    c = P.Solver(cfg)
    b.set_tiles(fftx=2048, fftz=1024, thomas=3, slab=5, expl=128, corr=64, cn=64, cnslab=0)
    c.set_tiles(cn=512, cnslab=0)
    a.set_tiles(cnslab=0)
    assert c.tiles()["cn"] == 512
    a.step(9)
    b.step(9)
    c.step(9)
    for k in FIELDS:
        ref = a.get_field(k).cpu()
        assert torch.equal(ref, b.get_field(k).cpu()), k
        assert torch.equal(ref, c.get_field(k).cpu()), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_identical_runs_are_bitwise_reproducible(P, precision):
    """Every reduction (the adaptive dt, run statistics, diagnostics, ion flux,
    KE budget) combines partial sums in a fixed order, without atomics: two
    runs of one configuration agree bit for bit, fields and reductions alike."""
    import torch
    cfg = small(P, nx=48, ny=33, nz=36, dt=0.0, cfl=0.5, re=1500.0, vhat=12.0, debye=0.08, seed=21,
                u_noise=0.2, migration_face=2, precision=precision)
    note(f"case: two identical runs 48x33x36 {precision}, migration face 2")
    out = []
    for _ in range(2):
        g = P.Solver(cfg)
        g.stats_begin(1)
        g.step(60)
        g.sync()
        st = g.stats_read()
        out.append({"fields": {k: g.get_field(k).cpu() for k in FIELDS}, "clock": g.clock(), "stats": st,
                    "diag": g.diagnostics(), "flux": g.ion_flux(), "energy": g.energy_budget(),
                    "tau": g.wall_shear_stress()})
    a, b = out
    for k in FIELDS:
        assert torch.equal(a["fields"][k], b["fields"][k]), k
    assert a["clock"] == b["clock"] and a["diag"] == b["diag"] and a["energy"] == b["energy"]
    assert a["tau"] == b["tau"]
    assert a["stats"][0] == b["stats"][0] and a["stats"][1] == b["stats"][1] and a["stats"][2] == b["stats"][2]
    assert list(a["flux"][0]) == list(b["flux"][0]) and list(a["flux"][1]) == list(b["flux"][1])
    assert a["flux"][2:] == b["flux"][2:]
