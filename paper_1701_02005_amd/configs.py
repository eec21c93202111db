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
