"""Pins of the run-statistics reference (CPU only): the time-averaged plane
moments, RMS profiles and wall quantities behind the statistics of Sec. III.

  * exact laminar Couette flow (no noise, no voltage): the averaged velocity
    is the linear profile at the cell centres, its RMS is zero, both wall
    stresses are 1/Re, c_f = 2/Re, Re_tau = sqrt(Re) and u+ = y+ exactly
    (the viscous law of the wall holds across the whole laminar gap);
  * plane moments of a field a_j + b cos(2 pi i / nx) are exactly a_j and
    a_j^2 + b^2 / 2 on the discrete grid, and a row-dependent mean catches
    an average over the wrong axes;
  * time weights are the time since the previous sample (hand-computed
    numbers), and RMS includes fluctuations in time.
"""
import math

import numpy as np
import pytest

from oracle import stats_oracle as S


def _fields(M=5, nz=4, nx=6, **over):
    f = {k: np.zeros((M, nz, nx)) for k in S.FIELDS}
    f.update(over)
    return f


def test_plane_moments_of_a_cosine():
    M, nz, nx = 5, 4, 6
    a = np.linspace(-1.0, 2.0, M)
    b = 0.7
    i = np.arange(nx)
    u = a[:, None, None] + b * np.cos(2 * np.pi * i / nx)[None, None, :] + 0.0 * np.zeros((M, nz, nx))
    k = np.arange(nz)
    w = 3.0 + 0.5 * np.sin(2 * np.pi * k / nz)[None, :, None] + np.zeros((M, nz, nx))
    m = S.plane_moments(_fields(u=u, w=w))
    assert m.shape == (14, M)
    assert np.allclose(m[0], a, atol=1e-14)
    assert np.allclose(m[7], a ** 2 + b ** 2 / 2, atol=1e-14)
    assert np.allclose(m[2], 3.0, atol=1e-14)
    assert np.allclose(m[9], 9.0 + 0.25 / 2, atol=1e-14)
    assert np.allclose(S.rms(m[0], m[7]), b / math.sqrt(2.0), atol=1e-12)
    # the other fields are zero
    assert np.all(m[[1, 3, 4, 5, 6, 8, 10, 11, 12, 13]] == 0.0)


def test_time_weights_are_the_elapsed_time():
    ta = S.TimeAverage(t0=0.0)
    ta.sample(1.0, _fields(cp=np.full((5, 4, 6), 2.0)))
    ta.sample(3.0, _fields(cp=np.full((5, 4, 6), 5.0)))
    avg = ta.averages()
    assert ta.time == 3.0 and ta.samples == 2
    # weights 1 and 2: (1*2 + 2*5)/3 = 4 (equal weights would give 3.5)
    assert np.allclose(avg[3], 4.0, atol=1e-15)
    assert np.allclose(avg[10], (1 * 4 + 2 * 25) / 3.0, atol=1e-14)


def test_rms_includes_fluctuations_in_time():
    ta = S.TimeAverage(t0=10.0)
    for n in range(4):
        ta.sample(10.0 + 0.5 * (n + 1), _fields(phi=np.full((5, 4, 6), 1.0 if n % 2 == 0 else -1.0)))
    avg = ta.averages()
    assert np.allclose(avg[5], 0.0, atol=1e-15)
    assert np.allclose(S.rms(avg[5], avg[12]), 1.0, atol=1e-15)


@pytest.fixture
def couette(oracle_mod):
    oracle_mod.set_threads(1)
    o = oracle_mod.Oracle(nx=4, ny=17, nz=4, re=250.0, debye=0.1, vhat=0.0, dt=2e-3, stretch=1.5)
    o.init(0, 0.0, 0.0)
    yield o
    oracle_mod.set_threads(8)


def test_laminar_couette_statistics_are_exact(couette):
    o = couette
    ta = S.TimeAverage(o.t)
    for _ in range(9):
        o.substep()
        ta.sample(o.t, o.state())
    avg = ta.averages()
    yc, yn, re = o.yc, o.yn, 250.0
    assert np.allclose(avg[0], yc, atol=1e-13)
    assert np.allclose(S.rms(avg[0], avg[7]), 0.0, atol=1e-7)
    assert np.allclose(avg[3], 1.0, atol=1e-13) and np.allclose(avg[4], 1.0, atol=1e-13)
    assert np.allclose(avg[5], 0.0, atol=1e-13)
    wq = S.wall_quantities(avg[0], yn, re, -1.0, 1.0)
    assert abs(wq["tau_bottom"] - 1 / re) < 1e-12 and abs(wq["tau_top"] - 1 / re) < 1e-12
    assert abs(wq["cf"] - 2 / re) < 1e-12 and abs(wq["re_tau"] - math.sqrt(re)) < 1e-9
    yp, up = S.wall_units(avg[0], yc, re, -1.0, wq["tau_bottom"])
    assert np.allclose(up, yp, rtol=1e-11)
    assert abs(ta.time - o.t) < 1e-15 and ta.samples == 9
