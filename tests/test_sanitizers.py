"""Host sanitizer runs (CPU only): the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer runs a set of its pins, and the GPU library built
with AddressSanitizer on its host code only (the device code is unchanged)
runs its configuration checks, layout and grid tables, each in a child
process with the checker's runtime preloaded.  Any report fails the test."""
import glob
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CHILD_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
             "OMP_NUM_THREADS": "4"}


def _run(cmd, env_extra, timeout):
    env = dict(os.environ, **CHILD_ENV, **env_extra)
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = res.stdout + res.stderr
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert marker not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    return out


def test_oracle_pins_under_address_and_undefined_behaviour_checks():
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's ASan runtime is not installed")
    lib = ROOT / "oracle" / "libnspnp_oracle_san.so"
    tmp = lib.with_suffix(".so.tmp")
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=c11", "-Wall", "-ffp-contract=off",
                    "-o", str(tmp), str(ROOT / "oracle" / "nspnp_oracle.c"), "-lm"], check=True)
    os.replace(tmp, lib)
    out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_oracle_operators.py",
                "tests/test_oracle_limited.py", "tests/test_oracle_hybrid.py", "tests/test_oracle_dt_and_flux.py"],
               {"LD_PRELOAD": libasan, "NSPNP_ORACLE_SANITIZE": "1"}, 900)
    assert " passed" in out and " failed" not in out, out[-2000:]


def test_library_host_code_under_address_checks(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    hipcc = "/opt/rocm/bin/hipcc"
    if not rt or not os.path.exists(hipcc):
        pytest.skip("hipcc or its ASan runtime is not installed")
    csrc = ROOT / "paper_1701_02005_amd" / "csrc"
    lib = tmp_path / "libnspnp_san.so"
    srcs = [str(csrc / f) for f in ("api.hip", "stencil.hip", "poisson.hip", "reduce.hip", "ensemble.hip", "mlp.hip",
                                    "noalloc.hip")]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Wno-unused-command-line-argument", "-Wno-unused-value",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-Xarch_host", "-shared-libasan", f"-I{ROOT / 'include'}", *srcs, "-o", str(lib)],
                   check=True, capture_output=True)
    script = f"""
import dataclasses
from pathlib import Path
import paper_1701_02005_amd.binding as B
B.LIB_PATH = Path({str(lib)!r})
import paper_1701_02005_amd as P
lib = B.load_library()
ok = P.configs.couette_small()
for cfg in (ok, dataclasses.replace(ok, ny=513), P.configs.couette_large(), P.configs.couette_turbulent(precision="mixed"),
            dataclasses.replace(ok, implicit_xz=1, migration_face=2)):
    assert P.workspace_bytes(cfg) > 0
    yn, yc = B.grid(cfg)
    assert len(yn) == cfg.ny and len(yc) == cfg.ny - 1
for bad in (dict(nx=30), dict(nz=7), dict(ny=4), dict(ny=514), dict(re=0.0), dict(debye=-1.0),
            dict(migration_face=3), dict(implicit_xz=3)):
    assert P.workspace_bytes(dataclasses.replace(ok, **bad)) == 0
    assert lib.nspnp_last_error()
print("host checks ok")
"""
    out = _run([sys.executable, "-c", script], {"LD_PRELOAD": rt[-1]}, 300)
    assert "host checks ok" in out
