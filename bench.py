"""Throughput of the NS-PNP Runge-Kutta substep on one MI355X.

One "step" is one Runge-Kutta substep of the whole hot path: explicit
right-hand sides, Crank-Nicolson wall-normal solves, pressure projection
(FFT x/z + Thomas in y), potential solve and (every third substep) the
adaptive time step.  Inputs are synthetic and seeded (laminar Couette profile
plus uniform noise) and resident in HBM before timing starts.

Prints ONE JSON line: Mpoint-substeps/s (points = nx * ny * nz, ny the
number of wall-normal nodes), the roofline of the dominant kernel measured
with HIP events on the solver's stream, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0


def kernel_bytes(cfg, name: str, launches: int, substeps: int) -> float:
    """Algorithmic (compulsory) HBM bytes of all launches of one kernel class.

    w = state word (8 FP64, 4 mixed); scratch and spectral buffers are FP64.
    Per cell: explicit_rhs reads the 7 state fields, reads H^{k-1} (stages 2
    and 3), writes H^k (stages 1 and 2) and the 5 Crank-Nicolson right-hand
    sides; cn_tridiag reads r and the field and writes the field (5 fields);
    the x transforms read or write one real FP64 value and one half spectrum
    (nx/2+1 complex per line of nx); z transforms and the mode Thomas solve
    read and write the half spectrum once; correct reads psi and updates
    u, v, w, p; divergence reads u, v, w and writes one FP64 value; charge
    reads c+, c- and writes one FP64 value.
    """
    w = 8 if cfg.precision == "fp64" else 4
    n = cfg.nx * cfg.nz * (cfg.ny - 1)
    spec = 16.0 * (cfg.nx // 2 + 1) / cfg.nx  # half-spectrum bytes per cell
    if name == "explicit_rhs":
        # stages cycle 1,2,3: H_old read on 2 of 3, H_new written on 2 of 3
        per = 7 * w + 40 + 5 * w * (2.0 / 3.0) + 5 * w * (2.0 / 3.0)
    elif name == "cn_tridiag":
        per = 5 * (8 + 2 * w)
    elif name == "divergence":
        per = 3 * w + 8
    elif name in ("fft_x_r2c", "fft_x_c2r"):
        per = 8 + spec
    elif name in ("fft_z_fwd", "fft_z_inv", "thomas_modes"):
        per = 2 * spec
    elif name == "correct":
        per = 8 + 8 * w
    elif name == "charge":
        per = 2 * w + 8
    elif name == "store_phi":
        per = 8 + w
    elif name == "dt":
        per = 5 * w
    else:
        per = 0.0
    return per * n * launches


def cpu_baseline(cfg, nsub: int = 3) -> dict:
    """The FP64 oracle as it stands, on all host cores, on a bounded sample."""
    from oracle import oracle as O
    threads = os.cpu_count() or 1
    O.set_threads(threads)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    t0 = time.perf_counter()
    o.run(nsub)
    el = time.perf_counter() - t0
    return {"value": cfg.points * nsub / el / 1e6, "unit": "Mpoint-substeps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{nsub} substeps (one full RK3 step) of the {cfg.nx}x{cfg.ny}x{cfg.nz} case from its "
                      f"seeded initial state, FP64, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="couette_turbulent")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the solver is a single-GPU build "
              "(a multi-GPU z-slab decomposition is designed, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1701_02005_amd as P

    cfg = P.configs.WORKLOADS[args.workload](precision=args.precision)
    print(f"[bench] workload {args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} {args.precision}", file=sys.stderr,
          flush=True)
    solver = P.Solver(cfg, device="cuda:0")
    stream = solver.stream
    solver.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} substeps done", file=sys.stderr, flush=True)

    # clean timed region
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    solver.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    print(f"[bench] timed {args.steps} substeps: {ms:.1f} ms", file=sys.stderr, flush=True)

    # same length again with HIP events around every kernel launch
    solver.profile_enable(True)
    start2, stop2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start2.record(stream)
    solver.step(args.steps)
    stop2.record(stream)
    torch.cuda.synchronize()
    ms_prof = start2.elapsed_time(stop2)
    prof = solver.profile_read()
    solver.profile_enable(False)
    diag = solver.diagnostics()
    tb, tt = solver.wall_shear_stress()

    kernels = {}
    total_bytes = 0.0
    for name, (kms, cnt) in prof.items():
        if cnt == 0:
            continue
        b = kernel_bytes(cfg, name, cnt, args.steps)
        total_bytes += b
        kernels[name] = {"ms_per_launch": kms / cnt, "launches": cnt, "share": kms / ms_prof,
                         "GBs": b / (kms * 1e-3) / 1e9 if kms > 0 else None}
    dom = max(kernels, key=lambda k: kernels[k]["share"])
    dom_ms, dom_cnt = prof[dom]
    dom_bytes = kernel_bytes(cfg, dom, dom_cnt, args.steps)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    per_launch_bytes = dom_bytes / dom_cnt

    traffic = None
    tr_file = ROOT / "profiles" / "traffic.json"
    if tr_file.exists():
        try:
            tr = json.loads(tr_file.read_text())
            key = f"{args.workload}/{args.precision}/{dom}"
            traffic = tr.get(key)
        except (ValueError, OSError):
            traffic = None

    value = cfg.points * args.steps / (ms * 1e-3) / 1e6
    out = {
        "metric": "Mpoint-substeps/s",
        "value": value,
        "unit": "Mpoint-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} Re={cfg.re:g} "
                               f"debye={cfg.debye:g} vhat={cfg.vhat:g} {args.precision}",
                   "points": cfg.points, "cells": cfg.cells, "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "avg_launch_ms": dom_ms / dom_cnt},
        "substep_roofline": {"algorithmic_GBs": total_bytes / (ms_prof * 1e-3) / 1e9,
                             "frac": total_bytes / (ms_prof * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "bytes_per_cell": total_bytes / (cfg.cells * args.steps)},
        "kernels": kernels,
        "profiled_region_ms": ms_prof,
        "state_check": {"tau_bottom": tb, "tau_top": tt, "max_div": diag["max_div"]},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
