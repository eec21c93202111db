"""Seeded synthetic inputs shared by the oracle and the GPU tests.

Holds no arithmetic of the method: only random arrays of given shapes and the
plane-Couette workload definitions (sizes and control parameters)."""
import numpy as np


def random_field(shape, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal(shape)


def parity(gpu, ref):
    """max |a - b| / max |b| (absolute when b is identically zero)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    err = np.max(np.abs(gpu - ref)) if ref.size else 0.0
    return err / den if den > 0 else err
