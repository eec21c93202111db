"""The statistics-campaign pipeline end to end on a small laminar case,
where the answer is closed-form: c_f = 2/Re, Re_tau = sqrt(Re), u+ = y+;
and its checkpoint/resume path continues the statistics exactly."""
import dataclasses
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02005_amd as pkg
    pkg.load_library()
    return pkg


def test_laminar_campaign_and_resume(P, tmp_path):
    from paper_1701_02005_amd import campaign as C
    cfg = dataclasses.replace(P.configs.couette_small(), vhat=0.0, u_noise=0.0, c_noise=0.0, dt=0.0, cfl=0.5)
    print("case: laminar campaign 32x33x32", flush=True)
    sys.stdout.flush()
    ck = tmp_path / "camp.ckpt"
    full = C.run_campaign(cfg, t_spin=0.5, t_avg=2.0, every=1, monitor=0.1, amp=0.0, ckpt=str(ck),
                          ckpt_every=1e9, log=lambda m: None)
    assert full["samples"] > 10 and full["averaged_time"] > 1.9
    assert abs(full["cf"] - 2.0 / cfg.re) < 1e-11
    assert abs(full["re_tau"] - math.sqrt(cfg.re)) < 1e-8
    assert np.allclose(full["u_plus"], full["y_plus"], rtol=1e-10)
    assert full["cf_stderr"] < 1e-12
    # a campaign stopped inside the averaging window and resumed from its
    # checkpoint reaches the same statistics
    part = C.run_campaign(cfg, t_spin=0.5, t_avg=1.0, every=1, monitor=0.1, amp=0.0, ckpt=str(ck),
                          ckpt_every=1e9, log=lambda m: None)
    rest = C.run_campaign(cfg, t_spin=0.5, t_avg=2.0, every=1, monitor=0.1, resume=str(ck), log=lambda m: None)
    assert rest["samples"] > part["samples"]
    assert abs(rest["cf"] - 2.0 / cfg.re) < 1e-11


def test_charged_laminar_campaign_with_limited_advection(P):
    """The sweep's path (migration_face 2, equilibrium double layer, charged
    walls) on laminar flow: the Coulomb force is wall-normal and balanced by
    the pressure, so c_f = 2/Re; the layer stays at the discrete equilibrium
    the host solved, and the ion RMS is zero."""
    from paper_1701_02005_amd import campaign as C
    cfg = dataclasses.replace(P.configs.couette_small(), nx=16, ny=33, nz=16, vhat=10.0, debye=0.1, sc=1.0,
                              migration_face=2, u_noise=0.0, c_noise=0.0, dt=0.0, cfl=0.5)
    print("case: charged laminar campaign 16x33x16, vhat 10, migration_face 2", flush=True)
    sys.stdout.flush()
    cp_eq, cm_eq, _ = C.equilibrium_ions(cfg)
    rep = C.run_campaign(cfg, t_spin=0.5, t_avg=1.0, every=1, monitor=0.1, amp=0.0, log=lambda m: None)
    assert rep["stopped"] is None
    assert abs(rep["cf"] - 2.0 / cfg.re) < 1e-9
    np.testing.assert_allclose(rep["mean"]["cp"], cp_eq, rtol=1e-7)
    np.testing.assert_allclose(rep["mean"]["cm"], cm_eq, rtol=1e-7)
    # (the RMS is sqrt(<q^2> - <q>^2): rounding of q^2 ~ 10^3 leaves ~1e-5 absolute)
    assert max(rep["rms"]["cp"]) < 1e-4 * max(cp_eq) and max(rep["rms"]["cm"]) < 1e-4 * max(cp_eq)
    assert set(rep["rms_peaks"]) == {"cp_lower", "cp_upper", "cm_lower", "cm_upper"}


def test_metrics_lines_on_laminar_flow(P, tmp_path):
    """The JSON-lines metrics of a laminar campaign: c_f = 2/Re, Re_tau =
    sqrt(Re), constant ion contents, a divergence-free field, a KE budget that
    closes (steady flow: wall work = dissipation, no Coulomb work) and the
    event profiler's per-class times."""
    import json
    from paper_1701_02005_amd import campaign as C
    cfg = dataclasses.replace(P.configs.couette_small(), vhat=0.0, u_noise=0.0, c_noise=0.0, dt=0.0, cfl=0.5)
    print("case: laminar campaign metrics 32x33x32", flush=True)
    sys.stdout.flush()
    path = tmp_path / "metrics.jsonl"
    C.run_campaign(cfg, t_spin=0.3, t_avg=0.6, every=1, monitor=0.1, amp=0.0, log=lambda m: None,
                   metrics=str(path), metrics_kernels=True)
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(recs) >= 8
    m0 = recs[0]["ion_content"]
    for r in recs:
        assert abs(r["cf"] - 2.0 / cfg.re) < 1e-11
        assert abs(r["re_tau"] - math.sqrt(cfg.re)) < 1e-8
        assert abs(r["ion_content"][0] - m0[0]) < 1e-12 * m0[0] and abs(r["ion_content"][1] - m0[1]) < 1e-12 * m0[1]
        assert r["max_div"] < 1e-12
        assert "explicit_rhs" in r["kernel_ms"] and r["kernel_ms"]["explicit_rhs"] > 0
    for r in recs[1:]:
        assert abs(r["budget_residual"]) < 1e-9 * r["energy"]["dissipation"]
