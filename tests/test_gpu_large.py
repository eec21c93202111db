"""The 512x385x512 case (~101 M points): the mixed-precision form against the
FP64 GPU path (itself tied to the oracle by the parity tests) after 300
substeps at CFL 0.5 from the same seeded state; mean wall shear stress within
1e-4, ion contents and divergence at their precision floors."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_large_case_mixed_vs_fp64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02005_amd as P
    res = {}
    for prec in ("fp64", "mixed"):
        cfg = P.configs.couette_large(precision=prec, seed=0)
        note(f"case: 512x385x512 {prec}, 300 substeps")
        g = P.Solver(cfg)
        _, _, mp0, mm0 = g.ion_flux()
        for chunk in range(3):
            g.step(100)
            g.sync()
            note(f"  {prec}: {100 * (chunk + 1)} substeps")
        tb, tt = g.wall_shear_stress()
        _, _, mp, mm = g.ion_flux()
        res[prec] = dict(tau=0.5 * (tb + tt), drift=max(abs(mp - mp0) / mp0, abs(mm - mm0) / mm0),
                         diag=g.diagnostics(), t=g.clock()[0])
        del g
        torch.cuda.empty_cache()
    a, b = res["mixed"], res["fp64"]
    rel = abs(a["tau"] - b["tau"]) / abs(b["tau"])
    note(f"mean wall shear: fp64 {b['tau']:.10e} mixed {a['tau']:.10e} rel {rel:.2e}; t = {b['t']:.4f}")
    note(f"ion content drift: fp64 {b['drift']:.2e}, mixed {a['drift']:.2e}; "
         f"max div: fp64 {b['diag']['max_div']:.2e}, mixed {a['diag']['max_div']:.2e}; "
         f"max |dPhi| {b['diag']['max_dphi']:.3f}")
    assert rel < 1e-4
    assert b["drift"] < 1e-12 and a["drift"] < 1e-5
    assert b["diag"]["max_div"] < 1e-10
    assert b["diag"]["min_cp"] > 0 and a["diag"]["min_cp"] > 0
