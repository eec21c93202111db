"""Throughput of the NS-PNP Runge-Kutta substep on one MI355X.

One "step" is one Runge-Kutta substep of the whole hot path: explicit
right-hand sides, Crank-Nicolson wall-normal solves, pressure projection
(FFT x/z + Thomas in y), potential solve and (every third substep) the
adaptive time step.  Inputs are synthetic and seeded (laminar Couette profile
plus uniform noise) and resident in HBM before timing starts.

Default workload: the large case, 512 x 385 x 512 (~101 M points), Re 6000,
Debye length 0.02, 20 thermal volts, in FP64 (the headline, the path held to
the oracle at 1e-10); the same workload in the mixed form (FP32 state and
stencils, FP64 solves and reductions) is measured the same way and reported
under "mixed" in the same line.

Prints ONE JSON line: Mpoint-substeps/s (points = nx * ny * nz, ny the
number of wall-normal nodes), the roofline of the dominant kernel measured
with HIP events on the solver's stream, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0


def kernel_bytes(cfg, name: str, launches: int, substeps: int) -> float:
    """Algorithmic (compulsory) HBM bytes of all launches of one kernel class
    inside the substep loop.

    w = state word (8 FP64, 4 mixed); spectral buffers and psi are FP64;
    s = 16 (nx/2+1)/nx bytes of half spectrum per cell.  Per cell and launch:
    explicit_rhs reads the 7 state fields, reads H^{k-1} on stages 2 and 3,
    writes H^k on stages 1 and 2 and the 5 Crank-Nicolson right-hand sides
    (state type); cn_tridiag reads r and the field and writes the field, 5
    fields.
    The pressure and potential solves run batched: fft_x_r2c reads u, v, w
    (divergence) and c+, c- (charge) and writes two half spectra; fft_z_*
    and thomas_modes read and write both half spectra once; fft_x_c2r reads
    them and writes psi (FP64) and phi (state); correct reads psi and
    updates u, v, w, p; dt (with the health check) reads u, v, w, c+, c-, phi
    once per three substeps.
    """
    w = 8 if cfg.precision == "fp64" else 4
    n = cfg.nx * cfg.nz * (cfg.ny - 1)
    sp = 16.0 * (cfg.nx // 2 + 1) / cfg.nx
    # limited advective face values of the ions (migration_face 2): the
    # correction pass reads u, v, w and c+-, updates the ions' r and (two
    # stages of three) their H
    lim = (3 * w + 2 * w + 2 * 2 * w + 2 * 2 * w * (2.0 / 3.0)) if getattr(cfg, "migration_face", 0) == 2 else 0.0
    per = {
        "explicit_rhs": 7 * w + 5 * w + 5 * w * (2.0 / 3.0) + 5 * w * (2.0 / 3.0) + lim,
        # implicit wall-normal diffusion: r and the field read, the field written; with the
        # three-direction factorisation x-lines (r in place), y (r in place), z-lines (q += x)
        "cn_tridiag": 5 * (7 if getattr(cfg, "implicit_xz", 0) else 3) * w,
        "fft_x_r2c": 5 * w + 2 * sp,
        # (with the fused y-march, fft_z_fwd and fft_z_inv are its two marches:
        # each reads and writes both half spectra once; the row-order c' table
        # the backward march reads is a precomputed pivot, not counted)
        "fft_z_fwd": 4 * sp,
        "thomas_modes": 4 * sp,
        "fft_z_inv": 4 * sp,
        "fft_x_c2r": 2 * sp + 8 + w,
        "correct": 8 + 8 * w,
        "dt": 6 * w,
        "stats": 7 * w,  # run statistics: one read of the seven fields per sample
    }.get(name, 0.0)
    return per * n * launches


def cpu_baseline(cfg, nsub: int = 0) -> dict:
    """The FP64 oracle as it stands, on all host cores, on a bounded sample:
    whole RK3 steps (one step, 3 substeps, of the 512x385x512 case: ~25 s
    on 16 cores; 12 substeps of 256x193x256), timed after its initial
    state is built."""
    from oracle import oracle as O
    if nsub <= 0:
        nsub = 3 * max(1, round(4 * 12_648_448 / cfg.points))
    threads = os.cpu_count() or 1
    O.set_threads(threads)
    o = O.Oracle(**cfg.oracle_kwargs())
    o.init(cfg.seed, cfg.u_noise, cfg.c_noise)
    t0 = time.perf_counter()
    o.run(nsub)
    el = time.perf_counter() - t0
    return {"value": cfg.points * nsub / el / 1e6, "unit": "Mpoint-substeps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{nsub} substeps ({nsub // 3} full RK3 steps) of the {cfg.nx}x{cfg.ny}x{cfg.nz} case from its "
                      f"seeded initial state, FP64, {el:.1f} s"}


def measure(cfg, args, P, torch, tiles_trial: int) -> dict:
    """Autotune (unless disabled), warm up, time args.steps substeps with HIP
    events on the solver's stream, then time the same length again with
    events around every kernel launch.  Returns the throughput, per-kernel
    table and the dominant kernel's roofline."""
    solver = P.Solver(cfg, device="cuda:0")
    stream = solver.stream
    tiles = None
    fixed = args.tiles.get(cfg.precision) if args.tiles else None
    if fixed:  # launch shapes given on the command line (e.g. those a timed run's tuner chose)
        solver.set_tiles(**fixed)
        tiles = solver.tiles()
        print(f"[bench] {cfg.precision}: launch shapes set to {tiles}", file=sys.stderr, flush=True)
    elif not args.no_autotune:  # launch shapes by the library's autotuner (advances the run)
        tiles = solver.autotune(None, tiles_trial)
        print(f"[bench] {cfg.precision}: autotuned launch shapes {tiles}", file=sys.stderr, flush=True)
    if args.stats_every > 0:
        solver.stats_begin(args.stats_every)
    if args.wall_amplitude:
        x = torch.arange(cfg.nx, dtype=torch.float64, device="cuda") * (cfg.lx / cfg.nx)
        z = torch.arange(cfg.nz, dtype=torch.float64, device="cuda") * (cfg.lz / cfg.nz)
        gw = args.wall_amplitude * torch.cos(2 * z)[:, None] * torch.cos(x)[None, :]
        solver.set_wall_potential(gw, -gw)
        solver.refresh_potential()
    solver.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] {cfg.precision}: warmup {args.warmup} substeps done", file=sys.stderr, flush=True)

    # clean timed region
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    solver.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    print(f"[bench] {cfg.precision}: timed {args.steps} substeps: {ms:.1f} ms", file=sys.stderr, flush=True)

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
    del solver
    torch.cuda.empty_cache()

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

    # HBM bytes per launch from the rocprofv3 counter runs, while the kernel
    # source they were taken from is unchanged
    traffic = None
    tr_file = ROOT / "profiles" / "traffic.json"
    # (counters were taken with the default face rules and without the x/z solves)
    if tr_file.exists() and not args.implicit_xz and not args.migration_face:
        try:
            from paper_1701_02005_amd import pmc_traffic
            ent = json.loads(tr_file.read_text()).get(f"{args.workload}/{cfg.precision}/{dom}")
            src = Path(ent["source"]).name if ent else None
            cn_slab = bool(tiles and tiles.get("cnslab"))
            z_fused = bool(tiles) and tiles.get("thomas") == 0
            same_kernels = ent and tuple(ent.get("kernels", ())) == tuple(
                pmc_traffic.class_kernels(dom, cn_slab, z_fused))
            if same_kernels and ent.get("source_sha256") == pmc_traffic.source_hash(src):
                traffic = ent["bytes_per_launch"]
        except (ValueError, OSError, KeyError):
            traffic = None
    return {
        "value": cfg.points * args.steps / (ms * 1e-3) / 1e6,
        "ms_per_step": ms / args.steps,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes/launch",
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "avg_launch_ms": dom_ms / dom_cnt},
        "substep_roofline": {"algorithmic_GBs": total_bytes / (ms_prof * 1e-3) / 1e9,
                             "frac": total_bytes / (ms_prof * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "bytes_per_cell": total_bytes / (cfg.cells * args.steps)},
        "kernels": kernels,
        "launch_shapes": tiles or "library defaults",
        "profiled_region_ms": ms_prof,
        "state_check": {"tau_bottom": tb, "tau_top": tt, "max_div": diag["max_div"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=15)
    ap.add_argument("--workload", default="couette_large")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64 for the single runs (the large case adds its mixed form to the "
                         "line), the ensemble's own (mixed) for 'ensemble'")
    ap.add_argument("--no-mixed", action="store_true",
                    help="large case: do not add the mixed form's measurement to the line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default launch shapes instead of the autotuned ones")
    ap.add_argument("--tiles", action="append", default=[],
                    help="PREC:name=value,... launch shapes of one precision (fp64 or mixed) instead of the "
                         "autotuner's, e.g. fp64:expl=256,slab=16,cnslab=32 (for profiler runs that must time "
                         "the shapes a timed run chose without the tuner's trial launches)")
    ap.add_argument("--stats-every", type=int, default=0,
                    help="also sample the run statistics every N substeps in the timed regions "
                         "(a separate measurement; the default line has no sampling)")
    ap.add_argument("--implicit-xz", action="store_true",
                    help="diffusion implicit in x and z too (three-direction approximate factorisation)")
    ap.add_argument("--migration-face", type=int, default=0, choices=[0, 1, 2],
                    help="face rules of the ion fluxes: 1 hybrid migration, 2 also limited advection "
                         "(a separate measurement of the positivity options)")
    ap.add_argument("--wall-amplitude", type=float, default=0.0,
                    help="time with a wall-potential pattern A cos(x) cos(2z) on both walls "
                         "(a separate measurement of the inhomogeneous potential solve)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before timing, run one plain device-to-device copy of this many MiB (a "
                         "reference kernel of known traffic for hardware byte counters)")
    args = ap.parse_args()
    tiles_by_prec = {}
    for spec in args.tiles:
        prec, _, kv = spec.partition(":")
        tiles_by_prec[prec] = {k: int(v) for k, v in (item.split("=") for item in kv.split(",") if item)}
    args.tiles = tiles_by_prec

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the solver is a single-GPU build "
              "(a multi-GPU z-slab decomposition is designed, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1701_02005_amd as P

    if args.workload == "ensemble":
        bench_ensemble(args, P, torch)
        return
    explicit_precision = args.precision is not None
    if args.precision is None:
        args.precision = "fp64"
    cfg = P.configs.WORKLOADS[args.workload](precision=args.precision)
    if args.implicit_xz:
        cfg = dataclasses.replace(cfg, implicit_xz=1)
    if args.migration_face:
        cfg = dataclasses.replace(cfg, migration_face=args.migration_face)
    print(f"[bench] workload {args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} {args.precision}", file=sys.stderr,
          flush=True)
    if args.copy_calibration_mb > 0:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nbytes} bytes read + {nbytes} bytes written", file=sys.stderr,
              flush=True)
        del src, dst
    # launch-shape trials: whole RK steps; 6 substeps suffice where one substep takes milliseconds
    trial = 6 if cfg.cells > 50_000_000 else 30
    res = measure(cfg, args, P, torch, trial)

    out = {
        "metric": "Mpoint-substeps/s",
        "value": res["value"],
        "unit": "Mpoint-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} Re={cfg.re:g} "
                               f"debye={cfg.debye:g} vhat={cfg.vhat:g} {args.precision}",
                   "points": cfg.points, "cells": cfg.cells, "precision": args.precision,
                   "parallelism": "single GPU", **({"stats_every": args.stats_every} if args.stats_every else {}),
                   **({"wall_amplitude": args.wall_amplitude} if args.wall_amplitude else {}),
                   **({"implicit_xz": 1} if args.implicit_xz else {}),
                   **({"migration_face": args.migration_face} if args.migration_face else {})},
        **{k: res[k] for k in ("roofline", "substep_roofline", "kernels", "launch_shapes", "profiled_region_ms",
                               "state_check")},
    }
    # the large case is also quoted in its mixed form (FP32 state and stencils,
    # FP64 solves and reductions): same measurement, extra keys of the line
    if args.workload == "couette_large" and not explicit_precision and not args.no_mixed:
        cm = dataclasses.replace(cfg, precision="mixed")
        print("[bench] mixed form of the same workload", file=sys.stderr, flush=True)
        rm = measure(cm, args, P, torch, trial)
        out["mixed"] = {"value": rm["value"], "unit": "Mpoint-substeps/s", "ms_per_step": rm["ms_per_step"],
                        "dtype": "f32+f64", "roofline": rm["roofline"], "substep_roofline": rm["substep_roofline"],
                        "kernels": rm["kernels"], "launch_shapes": rm["launch_shapes"],
                        "state_check": rm["state_check"]}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


def bench_ensemble(args, P, torch):
    """64 independent runs of uneven size (32 at 64x65x64, 32 at 48x49x48;
    Re, voltage and Debye length sampled per member), advanced together by
    graph replays of 30 substeps; timed with the library's default launch
    shapes and again after the autotuner has chosen them per size class."""
    prec = args.precision or "mixed"
    members = P.configs.ensemble_members(seed=0, precision=prec)
    points = sum(c.points for c in members)
    ens = P.Ensemble(members, device="cuda:0")
    steps = max(30, 30 * (args.steps // 30))
    print(f"[bench] ensemble of {len(members)} runs, {points} points, {prec}", file=sys.stderr, flush=True)

    def timed():
        ens.capture(30)
        ens.step(max(30, 30 * (args.warmup // 30)))
        ens.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ens.stream)
        ens.step(steps)
        b.record(ens.stream)
        ens.sync()
        return a.elapsed_time(b)

    ms_default = timed()
    print(f"[bench] default launch shapes: {steps} substeps in {ms_default:.1f} ms", file=sys.stderr, flush=True)
    tiles = ens.autotune(None, 6)
    ms_tuned = timed()
    print(f"[bench] tuned launch shapes: {steps} substeps in {ms_tuned:.1f} ms", file=sys.stderr, flush=True)
    value = points * steps / (ms_tuned * 1e-3) / 1e6
    out = {
        "metric": "Mpoint-substeps/s", "value": value, "unit": "Mpoint-substeps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": ms_tuned / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble 32 x 64x65x64 + 32 x 48x49x48 {prec}", "points": points,
                   "members": len(members), "parallelism": "single GPU, graph-replayed"},
        "default_shapes_value": points * steps / (ms_default * 1e-3) / 1e6,
        "autotune_gain": ms_default / ms_tuned,
        "tiles": tiles,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
