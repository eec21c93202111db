"""The HIP library loads and exports every symbol the public header declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "nspnp.h"
LIB = ROOT / "paper_1701_02005_amd" / "libnspnp.so"


def declared():
    return re.findall(r"NSPNP_API\s+[\w\s\*]*?\b(nspnp_\w+)\s*\(", HEADER.read_text())


def test_header_declares_the_boundary():
    names = set(declared())
    for n in ("nspnp_init_state", "nspnp_step", "nspnp_poisson_solve", "nspnp_wall_shear_stress",
              "nspnp_ion_flux"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not LIB.exists():
        pytest.skip("libnspnp.so not built")
    lib = ctypes.CDLL(str(LIB))
    for name in declared():
        assert hasattr(lib, name), name


def test_config_validation_without_gpu():
    if not LIB.exists():
        pytest.skip("libnspnp.so not built")
    import dataclasses
    import paper_1701_02005_amd as P
    ok = P.configs.couette_small()
    assert P.workspace_bytes(ok) > 0
    assert P.workspace_bytes(dataclasses.replace(ok, ny=513)) > 0
    for bad in (dict(nx=30), dict(nz=7), dict(ny=4), dict(ny=514), dict(re=0.0), dict(precision="fp64", debye=-1.0),
                dict(migration_face=3), dict(migration_face=-1), dict(implicit_xz=3)):
        assert P.workspace_bytes(dataclasses.replace(ok, **bad)) == 0
        assert P.load_library().nspnp_last_error()
