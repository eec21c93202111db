"""Thin ctypes binding of ``libnspnp.so`` (the C ABI in include/nspnp.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch provides the device memory (one workspace tensor per
solver) and the stream.  There is no CPU fallback: constructing a solver
without the built library or without a GPU raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, fields, asdict
from pathlib import Path
from typing import Dict, Tuple

import torch

LIB_PATH = Path(__file__).resolve().parent / "libnspnp.so"

FIELDS = {"u": 0, "v": 1, "w": 2, "cp": 3, "cm": 4, "phi": 5, "p": 6}
PREC = {"fp64": 0, "mixed": 1}

NSPNP_OK = 0
ERRORS = {-1: "invalid argument", -2: "unsupported size", -3: "HIP error", -4: "non-finite state",
          -5: "workspace"}


class NsPnpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nspnp error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class _CConfig(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("lx", ctypes.c_double), ("lz", ctypes.c_double), ("stretch", ctypes.c_double),
        ("re", ctypes.c_double), ("sc", ctypes.c_double), ("beta", ctypes.c_double),
        ("debye", ctypes.c_double), ("vhat", ctypes.c_double),
        ("u_top", ctypes.c_double), ("u_bot", ctypes.c_double), ("force_sign", ctypes.c_double),
        ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("u_noise", ctypes.c_double), ("c_noise", ctypes.c_double),
        ("implicit_xz", ctypes.c_int32), ("migration_face", ctypes.c_int32),
    ]


@dataclass
class Config:
    """Mirror of ``nspnp_config``; see include/nspnp.h for every field."""
    nx: int = 32
    ny: int = 33
    nz: int = 32
    precision: str = "fp64"
    lx: float = 6.283185307179586
    lz: float = 3.141592653589793
    stretch: float = 1.5
    re: float = 400.0
    sc: float = 1.0
    beta: float = 0.5
    debye: float = 0.1
    vhat: float = 5.0
    u_top: float = 1.0
    u_bot: float = -1.0
    force_sign: float = -1.0
    dt: float = 1e-3
    cfl: float = 0.5
    seed: int = 0
    u_noise: float = 0.01
    c_noise: float = 1e-3
    implicit_xz: int = 0  # 1: x/z diffusion implicit too (three-direction factorisation)
    migration_face: int = 0  # 1: hybrid (upwind where the potential jump across a face is >= 2);
    # 2: hybrid, and limited (van Leer) advective face values of the ions

    def to_c(self) -> _CConfig:
        c = _CConfig()
        for f in fields(self):
            val = getattr(self, f.name)
            if f.name == "precision":
                val = PREC[val]
            setattr(c, f.name, val)
        return c

    def oracle_kwargs(self) -> dict:
        """The same physical configuration as keyword arguments of the oracle."""
        d = asdict(self)
        for k in ("precision", "seed", "u_noise", "c_noise"):
            d.pop(k)
        return d

    @property
    def cells(self) -> int:
        return self.nx * self.nz * (self.ny - 1)

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def load_library() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(str(LIB_PATH))
    sig = {
        "nspnp_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_CConfig)]),
        "nspnp_init_state": (_I, [ctypes.POINTER(_CConfig), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "nspnp_step": (_I, [_P, ctypes.c_int32]),
        "nspnp_grid": (_I, [ctypes.POINTER(_CConfig), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "nspnp_poisson_solve": (_I, [_P, ctypes.c_int32, _P, _P]),
        "nspnp_wall_shear_stress": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "nspnp_ion_flux": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D),
                                ctypes.POINTER(_D)]),
        "nspnp_get_field": (_I, [_P, ctypes.c_int32, _P]),
        "nspnp_set_field": (_I, [_P, ctypes.c_int32, _P]),
        "nspnp_refresh_potential": (_I, [_P]),
        "nspnp_explicit_terms": (_I, [_P, ctypes.POINTER(_P)]),
        "nspnp_diagnostics": (_I, [_P, ctypes.POINTER(_D)]),
        "nspnp_get_clock": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64)]),
        "nspnp_set_clock": (_I, [_P, _D, _D, ctypes.c_int32, ctypes.c_int64]),
        "nspnp_sync": (_I, [_P]),
        "nspnp_stats_begin": (_I, [_P, ctypes.c_int32]),
        "nspnp_set_wall_potential": (_I, [_P, _P, _P]),
        "nspnp_stats_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D)]),
        "nspnp_save": (_I, [_P, ctypes.c_char_p]),
        "nspnp_autotune": (_I, [_P, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
        "nspnp_get_tiles": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "nspnp_set_tiles": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "nspnp_load": (_I, [_P, ctypes.c_char_p]),
        "nspnp_profile_enable": (_I, [_P, ctypes.c_int32]),
        "nspnp_profile_read": (_I, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_char_p),
                                    ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int64)]),
        "nspnp_destroy": (None, [_P]),
        "nspnp_last_error": (ctypes.c_char_p, []),
        "nspnp_ensemble_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_CConfig), ctypes.c_int32]),
        "nspnp_ensemble_init": (_I, [ctypes.POINTER(_CConfig), ctypes.c_int32, _P, ctypes.c_size_t, _P,
                                     ctypes.POINTER(_P)]),
        "nspnp_ensemble_step": (_I, [_P, ctypes.c_int32]),
        "nspnp_ensemble_sync": (_I, [_P]),
        "nspnp_ensemble_capture": (_I, [_P, ctypes.c_int32]),
        "nspnp_ensemble_stats": (_I, [_P, ctypes.c_int32]),
        "nspnp_ensemble_profiles": (_I, [_P, ctypes.c_int32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                         ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "nspnp_ensemble_get_field": (_I, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
        "nspnp_ensemble_set_field": (_I, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
        "nspnp_ensemble_refresh_potential": (_I, [_P, ctypes.c_int32]),
        "nspnp_ensemble_diagnostics": (_I, [_P, ctypes.c_int32, ctypes.POINTER(_D)]),
        "nspnp_ensemble_wall_shear_stress": (_I, [_P, ctypes.c_int32, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "nspnp_ensemble_ion_flux": (_I, [_P, ctypes.c_int32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                         ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "nspnp_ensemble_clock": (_I, [_P, ctypes.c_int32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                      ctypes.POINTER(ctypes.c_int64)]),
        "nspnp_ensemble_autotune": (_I, [_P, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
        "nspnp_ensemble_classes": (ctypes.c_int32, [_P]),
        "nspnp_ensemble_destroy": (None, [_P]),
        "nspnp_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
        "nspnp_mlp_init": (_I, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_float), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "nspnp_mlp_set_params": (_I, [_P, ctypes.POINTER(ctypes.c_float)]),
        "nspnp_mlp_get_params": (_I, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
        "nspnp_mlp_forward": (_I, [_P, _P, ctypes.c_int32, _P]),
        "nspnp_mlp_gradients": (_I, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
        "nspnp_mlp_train_step": (_I, [_P, _P, _P, ctypes.c_int32, ctypes.c_float, _P]),
        "nspnp_mlp_sync": (_I, [_P]),
        "nspnp_mlp_destroy": (None, [_P]),
        "nspnp_poisson_solve_noalloc": (_I, [ctypes.POINTER(_CConfig), ctypes.c_int32, _P, _P, _P]),
        "nspnp_stats_derived": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D),
                                     ctypes.POINTER(_D)]),
        "nspnp_energy_budget": (_I, [_P, ctypes.POINTER(_D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


DIAGNOSTIC_NAMES = ("ke", "max_div", "min_cp", "min_cm", "max_csum", "max_dphi")
STATS_FIELDS = ("u", "v", "w", "cp", "cm", "phi", "p")
STATS_NAMES = STATS_FIELDS + tuple(f + "2" for f in STATS_FIELDS)


def _check(rc: int):
    if rc != NSPNP_OK:
        raise NsPnpError(rc, load_library().nspnp_last_error().decode())


def grid(cfg: Config):
    """(node coordinates [ny], cell-centre coordinates [ny-1]) of the wall-normal grid."""
    c = cfg.to_c()
    yn, yc = (_D * cfg.ny)(), (_D * (cfg.ny - 1))()
    _check(load_library().nspnp_grid(ctypes.byref(c), yn, yc))
    return list(yn), list(yc)


def poisson_solve_noalloc(cfg: Config, kind: int, rhs: torch.Tensor, out: torch.Tensor | None = None,
                          stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """nspnp_poisson_solve_noalloc: the elliptic solve on cfg's grid with the
    library's fixed device scratch (no handle, no workspace).  rhs / out:
    contiguous float64 CUDA tensors of nx*nz*(ny-1) values."""
    n = cfg.cells
    for t in (rhs,) + (() if out is None else (out,)):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda" or t.numel() != n:
            raise ValueError("expected a contiguous float64 CUDA tensor of nx*nz*(ny-1) values")
    out = torch.empty_like(rhs) if out is None else out
    stream = stream if stream is not None else torch.cuda.current_stream(rhs.device)
    c = cfg.to_c()
    with torch.cuda.device(rhs.device):
        _check(load_library().nspnp_poisson_solve_noalloc(ctypes.byref(c), int(kind), ctypes.c_void_p(rhs.data_ptr()),
                                                          ctypes.c_void_p(out.data_ptr()),
                                                          ctypes.c_void_p(stream.cuda_stream)))
    return out


def workspace_bytes(cfg: Config) -> int:
    c = cfg.to_c()
    return int(load_library().nspnp_workspace_bytes(ctypes.byref(c)))


class Solver:
    """One NS-PNP state on one GPU.  Method names follow the C ABI."""

    def __init__(self, cfg: Config, device: str = "cuda:0", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("nspnp needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._c = cfg.to_c()
        nbytes = self.lib.nspnp_workspace_bytes(ctypes.byref(self._c))
        if nbytes == 0:
            raise NsPnpError(-1, self.lib.nspnp_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.M = cfg.ny - 1
        self.shape = (self.M, cfg.nz, cfg.nx)
        h = _P()
        with torch.cuda.device(self.device):
            _check(self.lib.nspnp_init_state(ctypes.byref(self._c), ctypes.c_void_p(self.workspace.data_ptr()),
                                             nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            try:
                self.lib.nspnp_sync(self._h)
            finally:
                self.lib.nspnp_destroy(self._h)
                self._h = None

    def _f64(self, t: torch.Tensor) -> torch.Tensor:
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device or t.numel() != self.M * self.cfg.nz * self.cfg.nx:
            raise ValueError("expected a contiguous float64 tensor of nx*nz*(ny-1) values on the solver's device")
        return t

    # ---- the C ABI -------------------------------------------------------
    def step(self, n_substeps: int = 1):
        _check(self.lib.nspnp_step(self._h, int(n_substeps)))

    def poisson_solve(self, kind: int, rhs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._f64(rhs)
        out = torch.empty_like(rhs) if out is None else self._f64(out)
        _check(self.lib.nspnp_poisson_solve(self._h, int(kind), ctypes.c_void_p(rhs.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr())))
        return out

    def wall_shear_stress(self) -> Tuple[float, float]:
        tb, tt = _D(), _D()
        _check(self.lib.nspnp_wall_shear_stress(self._h, ctypes.byref(tb), ctypes.byref(tt)))
        return tb.value, tt.value

    def ion_flux(self):
        n = self.cfg.ny
        jp, jm = (_D * n)(), (_D * n)()
        mp, mm = _D(), _D()
        _check(self.lib.nspnp_ion_flux(self._h, jp, jm, ctypes.byref(mp), ctypes.byref(mm)))
        return list(jp), list(jm), mp.value, mm.value

    def get_field(self, name: str) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.nspnp_get_field(self._h, FIELDS[name], ctypes.c_void_p(out.data_ptr())))
        return out

    def set_field(self, name: str, value: torch.Tensor):
        value = self._f64(value.contiguous())
        _check(self.lib.nspnp_set_field(self._h, FIELDS[name], ctypes.c_void_p(value.data_ptr())))
        self.sync()

    def refresh_potential(self):
        _check(self.lib.nspnp_refresh_potential(self._h))

    def explicit_terms(self) -> Dict[str, torch.Tensor]:
        outs = [torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(5)]
        arr = (_P * 5)(*[o.data_ptr() for o in outs])
        _check(self.lib.nspnp_explicit_terms(self._h, arr))
        return dict(zip(("u", "v", "w", "cp", "cm"), outs))

    def diagnostics(self) -> Dict[str, float]:
        """Kinetic energy, max |div u|, min c+, min c-, max(c+ + c-) and the
        largest potential difference across one cell face (max_dphi)."""
        out = (_D * 6)()
        _check(self.lib.nspnp_diagnostics(self._h, out))
        return dict(zip(DIAGNOSTIC_NAMES, list(out)))

    def clock(self):
        t, dt, st, ns = _D(), _D(), ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib.nspnp_get_clock(self._h, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(st),
                                        ctypes.byref(ns)))
        return t.value, dt.value, st.value, ns.value

    def set_clock(self, t: float, dt: float, stage: int, substeps: int):
        _check(self.lib.nspnp_set_clock(self._h, t, dt, int(stage), int(substeps)))

    def sync(self):
        """Waits for the queued work; NsPnpError(-4) once a health check has
        flagged the run."""
        _check(self.lib.nspnp_sync(self._h))

    def autotune(self, cache_path: str | None = None, trial_substeps: int = 6) -> Dict[str, int]:
        """Launch shapes chosen by timing (advances the run; results unchanged)."""
        out = (ctypes.c_int32 * len(Ensemble.TILE_NAMES))()
        path = cache_path.encode() if cache_path else None
        _check(self.lib.nspnp_autotune(self._h, path, int(trial_substeps), out))
        return dict(zip(Ensemble.TILE_NAMES, list(out)))

    def tiles(self) -> Dict[str, int]:
        out = (ctypes.c_int32 * len(Ensemble.TILE_NAMES))()
        _check(self.lib.nspnp_get_tiles(self._h, out))
        return dict(zip(Ensemble.TILE_NAMES, list(out)))

    def set_tiles(self, **changes):
        """Change launch shapes by name (e.g. cnslab=16)."""
        cur = self.tiles()
        for k, v in changes.items():
            if k not in cur:
                raise KeyError(k)
            cur[k] = int(v)
        arr = (ctypes.c_int32 * len(Ensemble.TILE_NAMES))(*[cur[k] for k in Ensemble.TILE_NAMES])
        _check(self.lib.nspnp_set_tiles(self._h, arr))

    def set_wall_potential(self, bot: torch.Tensor | None = None, top: torch.Tensor | None = None):
        """Wall values of phi [nz, nx] (float64, on the solver's device) on the
        lower / upper wall beyond -+vhat/2; None: zero."""
        ptrs = []
        self._wall_keep = []
        for g in (bot, top):
            if g is None:
                ptrs.append(None)
                continue
            g = g.to(device=self.device, dtype=torch.float64).contiguous()
            if g.numel() != self.cfg.nx * self.cfg.nz:
                raise ValueError("wall potential needs nz * nx values")
            self._wall_keep.append(g)
            ptrs.append(ctypes.c_void_p(g.data_ptr()))
        _check(self.lib.nspnp_set_wall_potential(self._h, ptrs[0], ptrs[1]))
        self.sync()  # the copies have left the caller's tensors

    def stats_begin(self, every: int = 1):
        """Clear the run statistics and sample every `every` substeps (0 stops)."""
        _check(self.lib.nspnp_stats_begin(self._h, int(every)))

    def stats_read(self):
        """(averaged time span, samples, {name: [M] time average}) with names
        STATS_NAMES: plane means of u, v, w, cp, cm, phi, p and of their squares."""
        M = self.M
        t, n = _D(), ctypes.c_int64()
        out = (_D * (len(STATS_NAMES) * M))()
        _check(self.lib.nspnp_stats_read(self._h, ctypes.byref(t), ctypes.byref(n), out))
        vals = list(out)
        return t.value, n.value, {k: vals[q * M:(q + 1) * M] for q, k in enumerate(STATS_NAMES)}

    def statistics(self) -> Dict[str, object]:
        """Time-averaged profiles and wall quantities of the run statistics
        (nspnp_stats_read and nspnp_stats_derived): mean and RMS profiles, tau
        at both walls from the mean velocity, c_f, Re_tau, u_tau and the mean
        velocity in wall units of the lower wall (NaN before the first sample)."""
        T, n, st = self.stats_read()
        M = self.M
        out, rms, yp, up = (_D * 6)(), (_D * (len(STATS_FIELDS) * M))(), (_D * M)(), (_D * M)()
        _check(self.lib.nspnp_stats_derived(self._h, out, rms, yp, up))
        yn, yc = grid(self.cfg)
        r = list(rms)
        return {
            "time": T, "samples": n, "yc": yc, "yn": yn[:M],
            "mean": {f: st[f] for f in STATS_FIELDS},
            "rms": {f: r[q * M:(q + 1) * M] for q, f in enumerate(STATS_FIELDS)},
            "tau_bottom": out[0], "tau_top": out[1], "tau": out[2], "cf": out[3], "re_tau": out[4],
            "u_tau": out[5], "y_plus": list(yp), "u_plus": list(up),
        }

    def energy_budget(self) -> Dict[str, float]:
        """Kinetic-energy budget terms (nspnp_energy_budget): dKE/dt =
        wall_work - dissipation + force_work."""
        out = (_D * 3)()
        _check(self.lib.nspnp_energy_budget(self._h, out))
        return dict(zip(("wall_work", "dissipation", "force_work"), list(out)))

    def save(self, path: str):
        """Checkpoint (fields, H buffers, clock, run statistics) to a file."""
        _check(self.lib.nspnp_save(self._h, str(path).encode()))

    def load(self, path: str):
        """Restore a checkpoint written for the same configuration."""
        _check(self.lib.nspnp_load(self._h, str(path).encode()))

    def profile_enable(self, on: bool = True):
        _check(self.lib.nspnp_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> Dict[str, Tuple[float, int]]:
        """{kernel class: (total ms, launches)} since profile_enable."""
        n = ctypes.c_int32()
        names = (ctypes.c_char_p * 16)()
        ms = (_D * 16)()
        cnt = (ctypes.c_int64 * 16)()
        _check(self.lib.nspnp_profile_read(self._h, ctypes.byref(n), names, ms, cnt))
        return {names[k].decode(): (ms[k], cnt[k]) for k in range(n.value)}


class Ensemble:
    """Independent runs advanced together (nspnp_ensemble_* calls).

    Work is queued on a dedicated stream of default priority (the legacy
    null stream cannot be captured into a graph); every call that returns
    data synchronises that stream."""

    TILE_NAMES = ("expl", "cn", "fftx", "fftz", "thomas", "corr", "slab", "cnslab")

    def __init__(self, cfgs, device: str = "cuda:0"):
        if not torch.cuda.is_available():
            raise RuntimeError("nspnp needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.cfgs = list(cfgs)
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        arr = (_CConfig * len(self.cfgs))(*[c.to_c() for c in self.cfgs])
        self._arr = arr
        nbytes = self.lib.nspnp_ensemble_workspace_bytes(arr, len(self.cfgs))
        if nbytes == 0:
            raise NsPnpError(-1, self.lib.nspnp_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = _P()
        _check(self.lib.nspnp_ensemble_init(arr, len(self.cfgs), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.nspnp_ensemble_destroy(self._h)
            self._h = None

    def __len__(self):
        return len(self.cfgs)

    def sync(self):
        """Waits for every member; NsPnpError(-4) once a health check has
        flagged a member."""
        _check(self.lib.nspnp_ensemble_sync(self._h))

    def step(self, n_substeps: int):
        _check(self.lib.nspnp_ensemble_step(self._h, int(n_substeps)))

    def capture(self, substeps_per_replay: int):
        _check(self.lib.nspnp_ensemble_capture(self._h, int(substeps_per_replay)))

    def stats(self, on: bool):
        _check(self.lib.nspnp_ensemble_stats(self._h, 1 if on else 0))

    def profiles(self, member: int):
        m = self.cfgs[member].ny - 1
        u, r, p = (_D * m)(), (_D * m)(), (_D * m)()
        wt = _D()
        _check(self.lib.nspnp_ensemble_profiles(self._h, member, u, r, p, ctypes.byref(wt)))
        return list(u), list(r), list(p), wt.value

    def get_field(self, member: int, name: str) -> torch.Tensor:
        c = self.cfgs[member]
        out = torch.empty((c.ny - 1, c.nz, c.nx), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(self.lib.nspnp_ensemble_get_field(self._h, member, FIELDS[name], ctypes.c_void_p(out.data_ptr())))
        self.sync()
        return out

    def set_field(self, member: int, name: str, value: torch.Tensor):
        c = self.cfgs[member]
        if value.dtype != torch.float64 or not value.is_contiguous() or value.numel() != c.cells:
            raise ValueError("expected a contiguous float64 tensor of nx*nz*(ny-1) values")
        torch.cuda.synchronize(self.device)
        _check(self.lib.nspnp_ensemble_set_field(self._h, member, FIELDS[name], ctypes.c_void_p(value.data_ptr())))
        self.sync()

    def diagnostics(self, member: int) -> Dict[str, float]:
        """Raises NsPnpError(-4) when the member's state is not finite."""
        out = (_D * 6)()
        _check(self.lib.nspnp_ensemble_diagnostics(self._h, member, out))
        return dict(zip(DIAGNOSTIC_NAMES, list(out)))

    def refresh_potential(self, member: int):
        _check(self.lib.nspnp_ensemble_refresh_potential(self._h, member))

    def wall_shear_stress(self, member: int):
        tb, tt = _D(), _D()
        _check(self.lib.nspnp_ensemble_wall_shear_stress(self._h, member, ctypes.byref(tb), ctypes.byref(tt)))
        return tb.value, tt.value

    def ion_flux(self, member: int):
        n = self.cfgs[member].ny
        jp, jm = (_D * n)(), (_D * n)()
        mp, mm = _D(), _D()
        _check(self.lib.nspnp_ensemble_ion_flux(self._h, member, jp, jm, ctypes.byref(mp), ctypes.byref(mm)))
        return list(jp), list(jm), mp.value, mm.value

    def clock(self, member: int):
        t, dt, ns = _D(), _D(), ctypes.c_int64()
        _check(self.lib.nspnp_ensemble_clock(self._h, member, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(ns)))
        return t.value, dt.value, ns.value

    def classes(self) -> int:
        return int(self.lib.nspnp_ensemble_classes(self._h))

    def autotune(self, cache_path: str | None = None, trial_substeps: int = 6):
        nc = self.classes()
        k = len(self.TILE_NAMES)
        out = (ctypes.c_int32 * (k * nc))()
        path = cache_path.encode() if cache_path else None
        _check(self.lib.nspnp_ensemble_autotune(self._h, path, int(trial_substeps), out))
        return [dict(zip(self.TILE_NAMES, list(out)[k * c: k * c + k])) for c in range(nc)]


class Mlp:
    """BF16 matrix-core surrogate network (nspnp_mlp_* calls).  Parameters
    cross as one flat FP32 array: W_0 [in x out] row-major, b_0, W_1, b_1..."""

    def __init__(self, sizes, max_rows: int, params, device: str = "cuda:0"):
        import numpy as np
        if not torch.cuda.is_available():
            raise RuntimeError("nspnp needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.sizes = [int(x) for x in sizes]
        self.nl = len(self.sizes) - 1
        self.max_rows = int(max_rows)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self._sz = (ctypes.c_int32 * len(self.sizes))(*self.sizes)
        self.nparams = sum(a * b + b for a, b in zip(self.sizes[:-1], self.sizes[1:]))
        nbytes = self.lib.nspnp_mlp_workspace_bytes(self.nl, self._sz, self.max_rows)
        if nbytes == 0:
            raise NsPnpError(-1, self.lib.nspnp_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.nparams
        h = _P()
        _check(self.lib.nspnp_mlp_init(self.nl, self._sz, self.max_rows,
                                       p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.nspnp_mlp_sync(self._h)
            self.lib.nspnp_mlp_destroy(self._h)
            self._h = None

    @staticmethod
    def _dev(t):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError("expected a contiguous float32 CUDA tensor")
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(self.lib.nspnp_mlp_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        import numpy as np
        p = np.zeros(self.nparams, dtype=np.float32)
        g = np.zeros(self.nparams, dtype=np.float32)
        _check(self.lib.nspnp_mlp_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p, g

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        out = torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device=self.device)
        _check(self.lib.nspnp_mlp_forward(self._h, self._dev(x), int(x.shape[0]), self._dev(out)))
        return out

    def gradients(self, x: torch.Tensor, y: torch.Tensor) -> float:
        loss = ctypes.c_float()
        _check(self.lib.nspnp_mlp_gradients(self._h, self._dev(x), self._dev(y), int(x.shape[0]),
                                            ctypes.byref(loss)))
        return loss.value

    def train_step(self, x: torch.Tensor, y: torch.Tensor, lr: float) -> torch.Tensor:
        _check(self.lib.nspnp_mlp_train_step(self._h, self._dev(x), self._dev(y), int(x.shape[0]), float(lr),
                                             self._dev(self._loss)))
        return self._loss

    def sync(self):
        _check(self.lib.nspnp_mlp_sync(self._h))
