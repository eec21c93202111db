"""Run statistics of the sheared-electrolyte runs, written out from their
plain definitions (arXiv:1701.02005, Sec. III: mean and RMS profiles across
the gap, friction coefficient and friction Reynolds number).

TEST INFRASTRUCTURE ONLY: the reference the GPU library's statistics are
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It imports nothing from the GPU
package.

Definitions (state arrays are [row j, z index k, x index i]):
- plane mean of q at row j: the arithmetic mean over the nx * nz points of
  the row; for v, row j is the node row below cell row j;
- a sample at time t adds w * (plane mean of q) and w * (plane mean of q^2)
  with w = t - (time of the previous sample, or of the start);
- the time average is the weighted sum divided by the sum of the weights;
- RMS profile: sqrt(<q^2> - <q>^2) of the time averages;
- wall shear stresses from the time-averaged velocity profile, as the viscous
  flux through the wall faces over the half cell next to each wall:
  tau_bottom = (u_0 - u_bot) / (Re dn_0 / 2), tau_top = (u_top - u_{M-1}) /
  (Re dn_{M-1} / 2); tau = mean of the two, c_f = 2 tau, Re_tau = Re sqrt(tau);
- wall units of the lower wall: u_tau = sqrt(tau_bottom), y+ = (1 + y) Re
  u_tau, u+ = (u - u_bot) / u_tau.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("u", "v", "w", "cp", "cm", "phi", "p")


def plane_moments(fields: dict) -> np.ndarray:
    """[14, M]: plane means of the seven fields, then of their squares."""
    means = [np.asarray(fields[f], dtype=np.float64).mean(axis=(1, 2)) for f in FIELDS]
    squares = [(np.asarray(fields[f], dtype=np.float64) ** 2).mean(axis=(1, 2)) for f in FIELDS]
    return np.array(means + squares)


class TimeAverage:
    """Time-weighted average of plane moments over samples."""

    def __init__(self, t0: float):
        self.t_last = float(t0)
        self.time = 0.0
        self.samples = 0
        self.acc = None

    def sample(self, t: float, fields: dict):
        w = float(t) - self.t_last
        m = plane_moments(fields)
        self.acc = w * m if self.acc is None else self.acc + w * m
        self.time += w
        self.t_last = float(t)
        self.samples += 1

    def averages(self) -> np.ndarray:
        if self.acc is None or self.time <= 0.0:
            return np.zeros((2 * len(FIELDS), 0))
        return self.acc / self.time


def rms(mean: np.ndarray, mean_sq: np.ndarray) -> np.ndarray:
    return np.sqrt(np.maximum(mean_sq - mean ** 2, 0.0))


def wall_quantities(u_mean: np.ndarray, yn: np.ndarray, re: float, u_bot: float, u_top: float) -> dict:
    M = len(u_mean)
    dn0, dn1 = yn[1] - yn[0], yn[M] - yn[M - 1]
    tau_b = (u_mean[0] - u_bot) / (re * 0.5 * dn0)
    tau_t = (u_top - u_mean[M - 1]) / (re * 0.5 * dn1)
    tau = 0.5 * (tau_b + tau_t)
    return {"tau_bottom": tau_b, "tau_top": tau_t, "tau": tau, "cf": 2.0 * tau, "re_tau": re * math.sqrt(abs(tau))}


def wall_units(u_mean: np.ndarray, yc: np.ndarray, re: float, u_bot: float, tau_bottom: float):
    ut = math.sqrt(abs(tau_bottom))
    return (1.0 + np.asarray(yc)) * re * ut, (np.asarray(u_mean) - u_bot) / ut
