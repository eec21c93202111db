"""The learned warm start, end to end at reduced size: a small ensemble run
until its double layers are stationary, the network trained on the GPU on
their profiles, and unseen parameter points started plain (laminar flow,
uniform ions) and warm (the network's profiles).  The double layer charges
on the time scale lam Re Sc, with a slower tail as the bulk gives up ions,
so the plain start's lower-half charge needs hundreds of time units to settle
within 1 %; the warm start begins close to the stationary charge.  Asserted
margin: warm t* at most three quarters of the plain t* at every point (the
three points measured at 0.46, 0.56 and 0.22 of it)."""
import dataclasses
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


RANGES = {"re": (100.0, 300.0), "vhat": (1.0, 6.0), "lnlam": (math.log(0.08), math.log(0.25))}


def runs(P, S, seed, n, **grid):
    base = P.binding.Config(nx=8, ny=33, nz=8, precision="mixed", re=200.0, sc=1.0, beta=0.5, debye=0.1, vhat=4.0,
                            dt=0.0, cfl=0.5, seed=seed, migration_face=1, **grid)
    return S.test_members(seed, n, base, RANGES)


def test_warm_start_reaches_stationary_charge_sooner():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02005_amd as P
    from paper_1701_02005_amd import surrogate as S
    train = runs(P, S, 5, 16)
    note(f"case: warm start, 16 training runs 8x33x8, Re {RANGES['re']}, vhat {RANGES['vhat']}")
    X, Y, y_t, info = S.ensemble_data(train, 24000, 3000, train[0], chunk=300, log=note)
    note(f"  {info['stationary']} of {info['members']} runs stationary in charge")
    assert info["stationary"] >= 12
    sizes = (3, 64, 64, 3 * train[0].ny)
    net, std, tr = S.train_network(X, Y, 2000, 2e-3, 0, sizes=sizes, ranges=RANGES, log=note)
    tests = runs(P, S, 6, 3)
    preds = S.predict(net, std, np.array([(c.re, c.vhat, c.debye) for c in tests]), ranges=RANGES)
    per, walls = S.compare_starts(tests, preds, y_t, t_end=1500.0, chunk=30, window=5.0, tol=0.01, log=note)
    for rec in per:
        assert "q" in rec, rec  # no start stopped by the health check
        q = rec["q"]
        assert not q["censored_plain"], rec
        assert not q["censored_warm"], rec
        assert q["t_warm"] <= 0.75 * q["t_plain"], rec
