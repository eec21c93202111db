"""ctypes binding of the FP64 CPU oracle (``nspnp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is what the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It imports nothing from the GPU package.

Every function mirrors one operator of the paper's method (arXiv:1701.02005,
Sec. II, Eqs. (1)-(4), Fig. 1); the C file documents each one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "nspnp_oracle.c"
_LIB = _HERE / "libnspnp_oracle.so"
# An instrumented (address and undefined-behaviour checking) build of the same
# source, made by the CPU sanitizer test, is loaded instead of the plain one
# when NSPNP_ORACLE_SANITIZE=1 (the process then has the checker's runtime
# preloaded)
_LIB_SAN = _HERE / "libnspnp_oracle_san.so"

FIELDS = {"u": 0, "v": 1, "w": 2, "cp": 3, "cm": 4, "phi": 5, "p": 6}


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fused multiply-add)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-ffp-contract=off", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_double), ("lz", ctypes.c_double), ("stretch", ctypes.c_double),
        ("re", ctypes.c_double), ("sc", ctypes.c_double), ("beta", ctypes.c_double),
        ("debye", ctypes.c_double), ("vhat", ctypes.c_double), ("u_top", ctypes.c_double),
        ("u_bot", ctypes.c_double), ("force_sign", ctypes.c_double), ("dt", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("implicit_xz", ctypes.c_int32), ("migration_face", ctypes.c_int32),
    ]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if os.environ.get("NSPNP_ORACLE_SANITIZE") == "1":
        if not _LIB_SAN.exists():
            raise RuntimeError(f"{_LIB_SAN} is not built (the CPU sanitizer test builds it)")
        path = _LIB_SAN
    else:
        if not _LIB.exists():
            build(force=False)
        path = _LIB
    lib = ctypes.CDLL(str(path))
    sig = {
        "or_create": (_P, [ctypes.POINTER(_Config)]),
        "or_destroy": (None, [_P]),
        "or_field": (_D, [_P, ctypes.c_int]),
        "or_hold": (_D, [_P, ctypes.c_int]),
        "or_yn": (_D, [_P]), "or_yc": (_D, [_P]), "or_dn": (_D, [_P]), "or_dc": (_D, [_P]),
        "or_time": (ctypes.c_double, [_P]),
        "or_get_dt": (ctypes.c_double, [_P]),
        "or_stage": (ctypes.c_int, [_P]),
        "or_set_clock": (None, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
        "or_coulomb_k": (ctypes.c_double, [ctypes.POINTER(_Config)]),
        "or_noise": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]),
        "or_splitmix_raw": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
        "or_fft": (None, [ctypes.c_int, _D, _D, ctypes.c_int]),
        "or_thomas": (None, [ctypes.c_int, _D, _D, _D, _D, _D]),
        "or_convection": (None, [_P, _D, _D, _D, _D, _D, _D]),
        "or_lap_xz": (None, [_P, _D, _D]),
        "or_coulomb": (None, [_P, _D, _D, _D, _D, _D, _D]),
        "or_ion_explicit": (None, [_P, _D, _D, _D, _D, _D, ctypes.c_double, _D]),
        "or_explicit_terms": (None, [_P, _D, _D, _D, _D, _D]),
        "or_divergence": (None, [_P, _D, _D, _D, _D]),
        "or_gradient": (None, [_P, _D, _D, _D, _D]),
        "or_apply_ly": (None, [_P, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]),
        "or_poisson": (None, [_P, ctypes.c_int, _D, _D]),
        "or_solve_potential": (None, [_P]),
        "or_refresh_potential": (None, [_P]),
        "or_set_wall_potential": (None, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "or_xz_solve": (None, [_P, ctypes.c_int, ctypes.c_double, _D]),
        "or_compute_dt": (ctypes.c_double, [_P]),
        "or_substep": (None, [_P]),
        "or_run": (None, [_P, ctypes.c_int]),
        "or_init": (None, [_P, ctypes.c_uint64, ctypes.c_double, ctypes.c_double]),
        "or_wall_shear": (None, [_P, _D, _D]),
        "or_ion_flux": (None, [_P, _D, _D, _D, _D]),
        "or_kinetic_energy": (ctypes.c_double, [_P]),
        "or_max_divergence": (ctypes.c_double, [_P]),
        "or_energy_terms": (None, [_P, _D, _D, _D]),
        "or_num_threads": (ctypes.c_int, []),
        "or_set_threads": (None, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


DEFAULTS = dict(lx=2 * np.pi, lz=np.pi, stretch=1.5, re=400.0, sc=1.0, beta=0.5, debye=0.1,
                vhat=5.0, u_top=1.0, u_bot=-1.0, force_sign=-1.0, dt=1e-3, cfl=0.5,
                nx=32, ny=33, nz=32, implicit_xz=0, migration_face=0)


def make_config(**kw) -> _Config:
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle config keys {sorted(unknown)}")
    d.update(kw)
    c = _Config()
    for k, v in d.items():
        setattr(c, k, int(v) if k in ("nx", "ny", "nz", "implicit_xz", "migration_face") else float(v))
    return c


def coulomb_k(**kw) -> float:
    c = make_config(**kw)
    return _load().or_coulomb_k(ctypes.byref(c))


def noise(seed: int, field: int, lin: int) -> float:
    return _load().or_noise(seed, field, lin)


def splitmix_raw(seed: int, n: int) -> int:
    return _load().or_splitmix_raw(seed, n)


def fft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised complex DFT of one line: sum_n x_n exp(sign 2 pi i k n / N)."""
    lib = _load()
    re = np.ascontiguousarray(np.real(x), dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(x), dtype=np.float64).copy()
    lib.or_fft(len(re), _ptr(re), _ptr(im), sign)
    return re + 1j * im


def thomas(a, b, c, d) -> np.ndarray:
    """Solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j (complex d)."""
    lib = _load()
    a, b, c = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c))
    dr = np.ascontiguousarray(np.real(d), dtype=np.float64).copy()
    di = np.ascontiguousarray(np.imag(d), dtype=np.float64).copy()
    lib.or_thomas(len(b), _ptr(a), _ptr(b), _ptr(c), _ptr(dr), _ptr(di))
    return dr + 1j * di


class Oracle:
    """One FP64 CPU NS-PNP solver instance."""

    def __init__(self, **kw):
        self._lib = _load()
        self.cfg = make_config(**kw)
        self._h = self._lib.or_create(ctypes.byref(self.cfg))
        if not self._h:
            raise ValueError("oracle: invalid configuration")
        self.nx, self.nz, self.ny = self.cfg.nx, self.cfg.nz, self.cfg.ny
        self.M = self.ny - 1
        self.shape = (self.M, self.nz, self.nx)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.or_destroy(self._h)
            self._h = None

    # ---- views -------------------------------------------------------
    def _view(self, ptr, n):
        return np.ctypeslib.as_array(ptr, shape=(n,))

    def field(self, name: str) -> np.ndarray:
        """Live view [M, nz, nx] of a state field (writes go to the solver)."""
        p = self._lib.or_field(self._h, FIELDS[name])
        return np.ctypeslib.as_array(p, shape=self.shape)

    def hold(self, q: int) -> np.ndarray:
        p = self._lib.or_hold(self._h, q)
        return np.ctypeslib.as_array(p, shape=self.shape)

    @property
    def yn(self):
        return self._view(self._lib.or_yn(self._h), self.M + 1).copy()

    @property
    def yc(self):
        return self._view(self._lib.or_yc(self._h), self.M).copy()

    @property
    def dn(self):
        return self._view(self._lib.or_dn(self._h), self.M).copy()

    @property
    def dc(self):
        return self._view(self._lib.or_dc(self._h), self.M + 1).copy()

    @property
    def dx(self):
        return self.cfg.lx / self.nx

    @property
    def dz(self):
        return self.cfg.lz / self.nz

    @property
    def t(self):
        return self._lib.or_time(self._h)

    @property
    def dt(self):
        return self._lib.or_get_dt(self._h)

    @property
    def stage(self):
        return self._lib.or_stage(self._h)

    def set_clock(self, t, dt, stage):
        self._lib.or_set_clock(self._h, t, dt, stage)

    def state(self) -> dict:
        return {k: self.field(k).copy() for k in FIELDS}

    def set_state(self, **fields):
        for k, v in fields.items():
            self.field(k)[...] = v

    # ---- method ------------------------------------------------------
    def init(self, seed: int, u_noise: float = 0.01, c_noise: float = 1e-3):
        self._lib.or_init(self._h, seed, u_noise, c_noise)

    def run(self, nsub: int):
        self._lib.or_run(self._h, nsub)

    def substep(self):
        self._lib.or_substep(self._h)

    def set_wall_potential(self, bot=None, top=None):
        """Wall values of phi [nz, nx] on the lower / upper wall (None: zero);
        used from the next potential solve on."""
        arrs = []
        for a in (bot, top):
            arrs.append(None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.nz, self.nx))
        self._wall = arrs  # keep the buffers alive for the call
        ptr = [None if a is None else _ptr(a) for a in arrs]
        self._lib.or_set_wall_potential(self._h, ptr[0], ptr[1])

    def xz_solve(self, d: int, beta: float, r: np.ndarray) -> np.ndarray:
        """(I - beta L_d)^-1 r along the periodic lines of direction d (0: x, 1: z)."""
        a = np.ascontiguousarray(r, dtype=np.float64).copy()
        self._lib.or_xz_solve(self._h, int(d), float(beta), _ptr(a))
        return a

    def solve_potential(self):
        self._lib.or_solve_potential(self._h)

    def compute_dt(self) -> float:
        return self._lib.or_compute_dt(self._h)

    def _new(self):
        return np.zeros(self.shape)

    def convection(self, u, v, w):
        cu, cv, cw = self._new(), self._new(), self._new()
        self._lib.or_convection(self._h, *map(_ptr, (np.ascontiguousarray(u), np.ascontiguousarray(v),
                                                     np.ascontiguousarray(w), cu, cv, cw)))
        return cu, cv, cw

    def lap_xz(self, q):
        out = self._new()
        self._lib.or_lap_xz(self._h, _ptr(np.ascontiguousarray(q)), _ptr(out))
        return out

    def coulomb(self, cp, cm, phi):
        fu, fv, fw = self._new(), self._new(), self._new()
        self._lib.or_coulomb(self._h, *map(_ptr, (np.ascontiguousarray(cp), np.ascontiguousarray(cm),
                                                  np.ascontiguousarray(phi), fu, fv, fw)))
        return fu, fv, fw

    def ion_explicit(self, u, v, w, c, phi, zs):
        out = self._new()
        args = [np.ascontiguousarray(a) for a in (u, v, w, c, phi)]
        self._lib.or_ion_explicit(self._h, *map(_ptr, args), float(zs), _ptr(out))
        return out

    def explicit_terms(self):
        hs = [self._new() for _ in range(5)]
        self._lib.or_explicit_terms(self._h, *map(_ptr, hs))
        return dict(zip(("u", "v", "w", "cp", "cm"), hs))

    def divergence(self, u=None, v=None, w=None):
        u = self.field("u") if u is None else np.ascontiguousarray(u)
        v = self.field("v") if v is None else np.ascontiguousarray(v)
        w = self.field("w") if w is None else np.ascontiguousarray(w)
        out = self._new()
        self._lib.or_divergence(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out))
        return out

    def gradient(self, psi):
        gx, gy, gz = self._new(), self._new(), self._new()
        self._lib.or_gradient(self._h, _ptr(np.ascontiguousarray(psi)), _ptr(gx), _ptr(gy), _ptr(gz))
        return gx, gy, gz

    def apply_ly(self, q, kind: int, qbot: float = 0.0, qtop: float = 0.0):
        """kind 0: zero-flux walls; 1: wall values (qbot, qtop); 2: node field."""
        out = self._new()
        self._lib.or_apply_ly(self._h, _ptr(np.ascontiguousarray(q)), kind, qbot, qtop, _ptr(out))
        return out

    def poisson(self, kind: int, rhs):
        out = self._new()
        self._lib.or_poisson(self._h, kind, _ptr(np.ascontiguousarray(rhs, dtype=np.float64)), _ptr(out))
        return out

    # ---- diagnostics -------------------------------------------------
    def wall_shear(self):
        tb, tt = ctypes.c_double(), ctypes.c_double()
        self._lib.or_wall_shear(self._h, ctypes.byref(tb), ctypes.byref(tt))
        return tb.value, tt.value

    def ion_flux(self):
        jp, jm = np.zeros(self.ny), np.zeros(self.ny)
        mp, mm = ctypes.c_double(), ctypes.c_double()
        self._lib.or_ion_flux(self._h, _ptr(jp), _ptr(jm), ctypes.byref(mp), ctypes.byref(mm))
        return jp, jm, mp.value, mm.value

    def kinetic_energy(self) -> float:
        return self._lib.or_kinetic_energy(self._h)

    def max_divergence(self) -> float:
        return self._lib.or_max_divergence(self._h)

    def energy_terms(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._lib.or_energy_terms(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value


def num_threads() -> int:
    return _load().or_num_threads()


def set_threads(n: int) -> None:
    """OpenMP thread count of subsequent oracle calls."""
    _load().or_set_threads(int(n))
