"""Synthetic plane-Couette workloads (sizes and control parameters only).

Geometry of the paper's runs (Sec. II): streamwise period 2 pi h, spanwise
period pi h, walls at y = +-1 moving at +-U, grid clustered at the walls.
Where the paper is silent the values below are stated readings: Sc = 1,
beta = 0.5 (the dilute-electrolyte value of Sec. II), tanh clustering 1.5,
"N thermal volts" across the walls means vhat = N.
"""
from __future__ import annotations

import math

from .binding import Config

TWO_PI = 2 * math.pi


def couette_small(precision: str = "fp64", seed: int = 0) -> Config:
    """32 x 33 x 32, Re 400, Debye length 0.1, 5 thermal volts, dt 1e-3."""
    return Config(nx=32, ny=33, nz=32, precision=precision, lx=TWO_PI, lz=math.pi, stretch=1.5, re=400.0,
                  sc=1.0, beta=0.5, debye=0.1, vhat=5.0, dt=1e-3, seed=seed)


def couette_turbulent(precision: str = "fp64", seed: int = 0) -> Config:
    """256 x 193 x 256, Re 3000, Debye length 0.05, 10 thermal volts, CFL 0.5."""
    return Config(nx=256, ny=193, nz=256, precision=precision, lx=TWO_PI, lz=math.pi, stretch=1.5, re=3000.0,
                  sc=1.0, beta=0.5, debye=0.05, vhat=10.0, dt=0.0, cfl=0.5, seed=seed)


def couette_large(precision: str = "mixed", seed: int = 0) -> Config:
    """512 x 385 x 512 (~101 M points), Re 6000, Debye length 0.02, 20 thermal volts."""
    return Config(nx=512, ny=385, nz=512, precision=precision, lx=TWO_PI, lz=math.pi, stretch=1.5, re=6000.0,
                  sc=1.0, beta=0.5, debye=0.02, vhat=20.0, dt=0.0, cfl=0.5, seed=seed)


WORKLOADS = {
    "couette_small": couette_small,
    "couette_turbulent": couette_turbulent,
    "couette_large": couette_large,
}


def ensemble_members(seed: int = 0, n_large: int = 32, n_small: int = 32, precision: str = "mixed"):
    """Uneven ensemble: n_large runs on 64 x 65 x 64 and n_small on 48 x 49 x 48.
    Member i draws (Re, vhat, Debye length) from a generator seeded with
    (seed, i): Re uniform on [500, 3000], vhat uniform on [0, 20], Debye
    length log-uniform on [0.02, 0.2]; Sc = 1, beta = 0.5, CFL 0.5."""
    import numpy as np
    members = []
    for i in range(n_large + n_small):
        rng = np.random.default_rng([seed, i])
        re = float(rng.uniform(500.0, 3000.0))
        vhat = float(rng.uniform(0.0, 20.0))
        lam = float(math.exp(rng.uniform(math.log(0.02), math.log(0.2))))
        n, ny = (64, 65) if i < n_large else (48, 49)
        members.append(Config(nx=n, ny=ny, nz=n, precision=precision, lx=TWO_PI, lz=math.pi, stretch=1.5, re=re,
                              sc=1.0, beta=0.5, debye=lam, vhat=vhat, dt=0.0, cfl=0.5, seed=seed * 1000 + i))
    return members
