"""HBM traffic per kernel launch from two rocprofv3 counter runs of bench.py.

rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE report, per dispatch, the
kilobytes the L2 fetched from and wrote to memory.  bench.py's calibration
copy (--copy-calibration-mb N: N MiB read and N MiB written by one
__amd_rocclr_copyBuffer dispatch) gives the factor that turns each counter
into bytes.  Each solver kernel class (the names of the library's event
profiler) is the sum of its HIP kernels' average per-dispatch traffic.

The result is merged into a JSON table keyed "workload/precision/class",
with the SHA-256 of the kernel source file, so that bench.py reports the
figure only while that source is unchanged.

    python -m paper_1701_02005_amd.pmc_traffic --fetch F.csv --write W.csv \\
        --copy-mb 1024 --workload couette_turbulent --precision fp64 \\
        --out profiles/traffic.json [--markdown]
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import re
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
CSRC = "paper_1701_02005_amd/csrc"

# profiler class -> (HIP kernels launched per class launch, source file)
CLASSES = {
    "dt": (("k_dt_partial", "k_dt_final"), "reduce.hip"),
    "explicit_rhs": (("k_explicit",), "stencil.hip"),
    "cn_tridiag": (("k_cn_coef", "k_cn_scan"), "stencil.hip"),  # lane-scan method
    "fft_x_r2c": (("k_fft_x_r2c",), "poisson.hip"),
    "fft_z_fwd": (("k_fft_z",), "poisson.hip"),
    "thomas_modes": (("k_thomas_tile",), "poisson.hip"),
    "fft_z_inv": (("k_fft_z",), "poisson.hip"),
    "fft_x_c2r": (("k_fft_x_c2r",), "poisson.hip"),
    "correct": (("k_correct",), "stencil.hip"),
}

# the same class under the row-slab Crank-Nicolson method (its first pass runs
# inside k_explicit; the scan across slabs and the apply pass remain)
CN_SLAB_KERNELS = ("k_cn_coef", "k_cn_slab_scan", "k_cn_slab_apply")


# the z transforms under the fused y-march method (mode-solve tile 0): the
# forward march (z transform + forward elimination) and the backward march
# (back-substitution + inverse z transform); no separate mode-solve kernel
Z_FUSED_KERNELS = {"fft_z_fwd": ("k_zthomas_fwd",), "fft_z_inv": ("k_zthomas_bwd",)}


def class_kernels(cls: str, cn_slab: bool = False, z_fused: bool = False):
    """HIP kernels that one launch of a profiler class runs."""
    if cls == "cn_tridiag" and cn_slab:
        return CN_SLAB_KERNELS
    if z_fused and cls in Z_FUSED_KERNELS:
        return Z_FUSED_KERNELS[cls]
    return CLASSES[cls][0]


def source_hash(fname: str) -> str:
    h = hashlib.sha256()
    h.update((ROOT / CSRC / fname).read_bytes())
    h.update((ROOT / CSRC / "internal.h").read_bytes())
    return h.hexdigest()


def kernel_key(name: str) -> str:
    """'void nspnp::(anonymous namespace)::k_explicit<double, 3>(...)' -> 'k_explicit'."""
    m = re.search(r"\b(k_[A-Za-z0-9_]+)", name)
    return m.group(1) if m else name


def load(path: Path):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[kernel_key(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per


def traffic(fetch_csv: Path, write_csv: Path, copy_mb: int):
    f, w = load(fetch_csv), load(write_csv)
    copy_kib = copy_mb * 1024.0
    ff = copy_kib / max(f["__amd_rocclr_copyBuffer"])
    fw = copy_kib / max(w["__amd_rocclr_copyBuffer"])
    per_kernel = {}
    for k in set(f) | set(w):
        if not k.startswith("k_"):
            continue
        fv, wv = f.get(k, [0.0]), w.get(k, [0.0])
        per_kernel[k] = (sum(fv) / len(fv) * ff * 1024.0, sum(wv) / len(wv) * fw * 1024.0, len(fv))
    return per_kernel, ff, fw


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True, type=Path)
    ap.add_argument("--write", required=True, type=Path)
    ap.add_argument("--copy-mb", type=int, default=1024)
    ap.add_argument("--workload", default="couette_turbulent")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--out", type=Path, default=ROOT / "profiles" / "traffic.json")
    ap.add_argument("--command", default="")
    ap.add_argument("--markdown", action="store_true")
    a = ap.parse_args(argv)
    per_kernel, ff, fw = traffic(a.fetch, a.write, a.copy_mb)
    table = json.loads(a.out.read_text()) if a.out.exists() else {}
    for cls, (kernels, src) in CLASSES.items():
        if cls == "cn_tridiag" and all(k in per_kernel for k in CN_SLAB_KERNELS):
            kernels = CN_SLAB_KERNELS
        if cls in Z_FUSED_KERNELS and all(k in per_kernel for k in Z_FUSED_KERNELS[cls]):
            kernels = Z_FUSED_KERNELS[cls]
        if not all(k in per_kernel for k in kernels):
            continue
        fb = sum(per_kernel[k][0] for k in kernels)
        wb = sum(per_kernel[k][1] for k in kernels)
        table[f"{a.workload}/{a.precision}/{cls}"] = {
            "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
            "kernels": list(kernels), "source": f"{CSRC}/{src}", "source_sha256": source_hash(src),
            "fetch_scale": ff, "write_scale": fw, "command": a.command,
        }
    a.out.write_text(json.dumps(table, indent=1, sort_keys=True) + "\n")
    if a.markdown:
        print(f"calibration: FETCH_SIZE x{ff:.4f}, WRITE_SIZE x{fw:.4f} (copy of {a.copy_mb} MiB)\n")
        print("| kernel | dispatches | fetch MiB | write MiB |")
        print("|---|---|---|---|")
        for k, (fb, wb, n) in sorted(per_kernel.items(), key=lambda kv: -(kv[1][0] + kv[1][1])):
            print(f"| {k} | {n} | {fb / 2**20:.1f} | {wb / 2**20:.1f} |")


if __name__ == "__main__":
    main()
