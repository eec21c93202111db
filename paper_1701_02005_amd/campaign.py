"""Statistics campaign of one sheared-electrolyte run (Sec. III): friction
coefficient, friction Reynolds number, mean velocity in wall units and RMS
profiles of the velocity, ion and potential fields, with error bars.

Pipeline (all GPU work through the HIP library):

1. start: the laminar Couette state of the configuration (ions in the
   zero-flow equilibrium double layer when the walls are charged) with a
   finite-amplitude disturbance (streamwise rolls, the streaks they carry and
   seeded noise; plane Couette flow is linearly stable, so small noise decays
   and turbulence needs such a trigger), or a checkpoint to resume from;
2. spin-up to t_spin, recording the plane-averaged wall shear stress of both
   walls every `monitor` time units;
3. averaging from t_spin to t_spin + t_avg with the library's run statistics
   (samples every `every` substeps, weighted by elapsed time), still
   recording the wall stress;
4. report: c_f = 2 tau and Re_tau = Re sqrt(tau) from the time-averaged mean
   velocity, their standard errors from batch means of the recorded stress
   history over the averaging window, u+(y+) at the lower wall and the RMS
   profiles.

Checkpoints (fields, H buffers, clock and the statistics sums) are written
every `ckpt_every` time units when a path is given; `--resume` continues a
campaign from one (the averaging phase resumes with its sums).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time
from pathlib import Path

import numpy as np

from . import configs
from .binding import Config, NsPnpError, Solver, grid

# values printed for the uncharged validation case (Re 3000, Sec. II); the
# two are not mutually consistent (Re sqrt(c_f / 2) = 159, not 172), so they
# are context for the measured numbers, not targets
PAPER_CF = 5.63e-3
PAPER_RE_TAU = 172.0

# control parameters of the paper's three charged cases (Sec. III, its table
# of simulation cases): Re 3000, Sc 3, h / lambda_D and beta as named
TABLE1 = {
    "L100": {"re": 3000.0, "sc": 3.0, "debye": 1.0 / 100.0, "beta": 0.5},
    "L100B": {"re": 3000.0, "sc": 3.0, "debye": 1.0 / 100.0, "beta": 1.5e-4},
    "L33": {"re": 3000.0, "sc": 3.0, "debye": 1.0 / 33.0, "beta": 0.5},
}


def perturbed_start(solver: Solver, amp: float, seed: int, beta: float = 4.0, alpha: float = 1.0):
    """Laminar state + disturbance of amplitude amp (fraction of the wall speed):
    rolls v = amp (1 - y^2)^2 cos(beta z) (1 + 0.3 sin(alpha x)) with the w that
    makes them divergence-free in (y, z), streaks u' = amp (1 - y^2) sin(beta z)
    (1 + 0.5 cos(alpha x)), and uniform noise of amplitude 0.05 amp on u, v, w
    (seeded).  The first substep's projection removes what divergence remains."""
    import torch
    cfg = solver.cfg
    dev = solver.device
    yn, yc = grid(cfg)
    Y = torch.tensor(yc, dtype=torch.float64, device=dev)[:, None, None]
    Yn = torch.tensor(yn[:-1], dtype=torch.float64, device=dev)[:, None, None]
    X = (torch.arange(cfg.nx, dtype=torch.float64, device=dev) * (cfg.lx / cfg.nx))[None, None, :]
    Z = (torch.arange(cfg.nz, dtype=torch.float64, device=dev) * (cfg.lz / cfg.nz))[None, :, None]
    gen = torch.Generator(device=dev).manual_seed(int(seed))
    shape = (cfg.ny - 1, cfg.nz, cfg.nx)

    def noise():
        return 0.1 * amp * (torch.rand(shape, generator=gen, device=dev, dtype=torch.float64) - 0.5)

    u = solver.get_field("u") + amp * (1 - Y ** 2) * torch.sin(beta * Z) * (1 + 0.5 * torch.cos(alpha * X)) + noise()
    v = amp * (1 - Yn ** 2) ** 2 * torch.cos(beta * Z) * (1 + 0.3 * torch.sin(alpha * X)) + noise()
    v[0] = 0.0  # the lower wall node
    w = amp * 4.0 * Y * (1 - Y ** 2) * torch.sin(beta * Z) / beta + noise()
    for name, f in (("u", u), ("v", v), ("w", w)):
        solver.set_field(name, f.contiguous())


def equilibrium_ions(cfg: Config):
    """Zero-flow equilibrium double layer of the discrete equations (the
    zero-shear stationary state, Sec. II): every interior face carries zero
    ion flux, so with the central face value of the migration flux each
    species' neighbour ratio is c_{j+1}/c_j = (1 -+ dPhi/2) / (1 +- dPhi/2)
    (dPhi = Phi_{j+1} - Phi_j, Phi = (vhat/2) y + phi); with the hybrid face
    value (migration_face = 1 or 2) faces with |dPhi| >= 2 take the upwind ratio
    1/(1 + z dPhi) (z dPhi > 0) or 1 - z dPhi instead.  Each species' content
    equals the gap volume (mean 1); phi solves the discrete potential equation
    with zero wall values.  Returns (c+, c-, phi) per cell row.  With the
    mean face value it needs |dPhi| < 2 across every face (positive ratios)."""
    from scipy.optimize import fsolve
    yn, yc = (np.asarray(a, dtype=np.float64) for a in grid(cfg))
    M = len(yc)
    dn = np.diff(yn)
    dc = np.concatenate([[yc[0] - yn[0]], np.diff(yc), [yn[M] - yc[M - 1]]])
    e0, lam = 0.5 * cfg.vhat, cfg.debye

    hybrid = getattr(cfg, "migration_face", 0) >= 1  # (advective face values play no part at zero velocity)

    def conc(phi, zs):
        dphi = e0 * dc[1:M] + np.diff(phi)
        ratio = (1 - zs * dphi / 2) / (1 + zs * dphi / 2)
        if hybrid:
            up = np.where(zs * dphi > 0, 1.0 / (1.0 + np.abs(dphi)), 1.0 + np.abs(dphi))
            ratio = np.where(np.abs(dphi) >= 2.0, up, ratio)
        c = np.concatenate([[1.0], np.cumprod(ratio)])
        return c * 2.0 / np.sum(c * dn)

    def residual(phi):
        flux = np.diff(np.concatenate([[0.0], phi, [0.0]])) / dc
        return np.diff(flux) / dn + (conc(phi, 1.0) - conc(phi, -1.0)) / (2 * lam ** 2)

    phi = fsolve(residual, np.zeros(M), xtol=1e-13, maxfev=50000)
    if np.max(np.abs(residual(phi))) > 1e-7 * max(1.0, 1.0 / lam ** 2):
        raise RuntimeError("equilibrium double layer: Newton solve did not converge")
    return conc(phi, 1.0), conc(phi, -1.0), phi


def set_equilibrium_ions(solver: Solver, vhat: float | None = None):
    """c+- of every plane set to the equilibrium double layer (of the run's
    vhat, or of the given wall voltage); phi re-solved."""
    import torch
    cfg = solver.cfg if vhat is None else dataclasses.replace(solver.cfg, vhat=vhat)
    cp, cm, _ = equilibrium_ions(cfg)
    shape = (solver.cfg.ny - 1, solver.cfg.nz, solver.cfg.nx)
    for name, prof in (("cp", cp), ("cm", cm)):
        t = torch.tensor(prof, dtype=torch.float64, device=solver.device)[:, None, None].expand(shape).contiguous()
        solver.set_field(name, t)
    solver.refresh_potential()


def batch_means(x: np.ndarray, nbatch: int = 10):
    """Mean of a correlated series and its standard error from nbatch
    contiguous batch means (the batches should be longer than the
    correlation time)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // nbatch
    if n < 1:
        return float(np.mean(x)) if len(x) else float("nan"), float("nan")
    b = x[: n * nbatch].reshape(nbatch, n).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbatch))


def metrics_record(s, prev: dict | None = None, kernels: bool = False) -> dict:
    """One line of run metrics from the library's reductions: clock, wall
    stresses with the instantaneous c_f = 2 tau and Re_tau = Re sqrt(tau)
    (tau the mean of both walls), ion contents, KE, max |div u|, the
    concentration minima, max |dPhi| and the KE-budget terms.  With the
    previous record, the budget residual dKE/dt - (wall work - dissipation +
    force work), the rate from the two records' KE and the mean of their
    terms (first order in the interval).  kernels: per-class ms per launch of
    the event profiler since the previous record (the profiler is on)."""
    t, dt, _, ns = s.clock()
    tb, tt = s.wall_shear_stress()
    _, _, mp, mm = s.ion_flux()
    d = s.diagnostics()
    eb = s.energy_budget()
    tau = 0.5 * (tb + tt)
    rec = {"t": t, "dt": dt, "substeps": int(ns), "tau_bottom": tb, "tau_top": tt, "cf": 2.0 * tau,
           "re_tau": s.cfg.re * math.sqrt(tau) if tau > 0 else float("nan"), "ion_content": [mp, mm],
           "ke": d["ke"], "max_div": d["max_div"], "min_c": [d["min_cp"], d["min_cm"]], "max_dphi": d["max_dphi"],
           "energy": eb}

    def net(e):
        return e["wall_work"] - e["dissipation"] + e["force_work"]

    if prev is not None and t > prev["t"]:
        rec["budget_residual"] = (d["ke"] - prev["ke"]) / (t - prev["t"]) - 0.5 * (net(eb) + net(prev["energy"]))
    if kernels:
        tot = s.profile_read()
        last = (prev or {}).get("_kernel_totals", {})
        rec["kernel_ms"] = {k: (ms - last.get(k, (0.0, 0))[0]) / max(1, n - last.get(k, (0.0, 0))[1])
                            for k, (ms, n) in tot.items() if n > last.get(k, (0.0, 0))[1]}
        rec["_kernel_totals"] = tot
    return rec


def run_campaign(cfg: Config, t_spin: float, t_avg: float, every: int = 10, monitor: float = 0.5,
                 amp: float = 0.3, seed: int = 7, ckpt: str | None = None, ckpt_every: float = 50.0,
                 resume: str | None = None, ion_start: str = "equilibrium", t_charge: float | None = None,
                 log=print, metrics: str | None = None, metrics_kernels: bool = False) -> dict:
    """t_charge (optional): the run starts uncharged (the configuration's
    vhat is applied as wall values -+vhat/2 of phi, a discretely identical
    form of the same walls, only from t_charge on, together with the
    equilibrium double layer); turbulence then develops before the double
    layer meets it.  Not combined with resume."""
    wall_v = 0.0
    if t_charge is not None:
        wall_v, cfg = cfg.vhat, dataclasses.replace(cfg, vhat=0.0)
    s = Solver(cfg)
    if resume:
        s.load(resume)
    else:
        if ion_start == "equilibrium" and cfg.vhat != 0.0:
            set_equilibrium_ions(s)  # the double layer forms on the gap's ion transit time otherwise
        perturbed_start(s, amp, seed)
    t0 = time.time()
    hist = []  # (t, tau_bottom, tau_top)
    mfile = open(metrics, "a") if metrics else None  # JSON lines, one per monitor interval
    if mfile and metrics_kernels:
        s.profile_enable(True)
    mprev = {"rec": None}
    st0 = s.clock()
    state = {"t": st0[0], "dt": st0[1], "ns": st0[3], "averaging": st0[0] >= t_spin, "next_ckpt": st0[0] + ckpt_every}
    if state["averaging"] and not resume:
        s.stats_begin(every)
    t_end = t_spin + t_avg

    charged = {"done": t_charge is None}

    def charge_walls():
        import torch
        plane = torch.ones((cfg.nz, cfg.nx), dtype=torch.float64, device=s.device)
        s.set_wall_potential(-0.5 * wall_v * plane, 0.5 * wall_v * plane)
        if ion_start == "equilibrium":
            set_equilibrium_ions(s, vhat=wall_v)
        else:
            s.refresh_potential()
        charged["done"] = True
        log(f"[campaign] walls charged to -+{wall_v / 2:g} at t = {state['t']:.2f}")

    def advance():
        while state["t"] < t_end:
            t, dt = state["t"], state["dt"]
            if not charged["done"] and t >= t_charge:
                charge_walls()
            if not state["averaging"] and t >= t_spin:
                s.stats_begin(every)
                state["averaging"] = True
                log(f"[campaign] statistics from t = {t:.2f}")
            target = min(t + monitor, t_spin if not state["averaging"] else t_end)
            # whole Runge-Kutta steps at the current dt (3 before the first dt exists)
            n = 3 if dt <= 0.0 else min(3000, max(3, 3 * int(math.ceil((target - t) / dt / 3.0))))
            s.step(n)
            t, dt, _, ns = s.clock()
            state.update(t=t, dt=dt, ns=ns)
            tb, tt = s.wall_shear_stress()
            hist.append((t, tb, tt))
            if mfile:
                rec = metrics_record(s, mprev["rec"], metrics_kernels)
                mprev["rec"] = rec
                mfile.write(json.dumps({k: v for k, v in rec.items() if not k.startswith("_")}) + "\n")
                mfile.flush()
            if ckpt and t >= state["next_ckpt"]:
                s.save(ckpt)
                state["next_ckpt"] = t + ckpt_every
            if len(hist) % 20 == 0:
                log(f"[campaign] t = {t:8.2f}  substeps = {ns}  tau = ({tb:.4e}, {tt:.4e})  "
                    f"wall {time.time() - t0:.1f} s")
        s.sync()
        if ckpt:
            s.save(ckpt)

    stopped = None
    try:
        advance()
    except NsPnpError as e:
        # the health check stopped the run (a non-finite value or a negative
        # concentration, checked once per Runge-Kutta step): the statistics
        # sampled before it are reported, flagged
        stopped = {"t": state["t"], "reason": str(e)}
        log(f"[campaign] stopped at t = {state['t']:.2f}: {e}")
    wall = time.time() - t0
    if mfile:
        mfile.close()
    st = s.statistics()
    if st["samples"] == 0:  # nothing averaged: no statistics to report
        for k in ("cf", "re_tau", "tau", "tau_bottom", "tau_top"):
            st[k] = float("nan")
    h = np.array(hist)
    avg_win = h[h[:, 0] > t_spin] if len(h) else h
    tau_series = 0.5 * (avg_win[:, 1] + avg_win[:, 2]) if len(avg_win) else np.array([])
    tau_mean, tau_se = batch_means(tau_series)
    cf_se = 2.0 * tau_se
    re_tau_se = cfg.re * 0.5 * tau_se / math.sqrt(abs(st["tau"])) if st["tau"] > 0 else float("nan")
    return {
        "rms_peaks": rms_peaks(st, cfg),
        "config": dataclasses.asdict(cfg), "ion_start": ion_start, "t_charge": t_charge, "wall_vhat": wall_v,
        "t_spin": t_spin, "t_avg": t_avg, "sample_every": every, "samples": st["samples"],
        "averaged_time": st["time"], "substeps": int(state["ns"]), "wall_s": wall, "stopped": stopped,
        "cf": st["cf"], "cf_stderr": cf_se, "re_tau": st["re_tau"], "re_tau_stderr": re_tau_se,
        "tau_bottom": st["tau_bottom"], "tau_top": st["tau_top"],
        "tau_history_mean": tau_mean, "laminar_cf": 2.0 / cfg.re,
        "paper_cf": PAPER_CF, "paper_re_tau": PAPER_RE_TAU,
        "y_plus": st["y_plus"], "u_plus": st["u_plus"], "yc": st["yc"],
        "mean": st["mean"], "rms": st["rms"],
        "tau_history": h.tolist(),
    }


def rms_peaks(st: dict, cfg) -> dict:
    """Position of the largest RMS fluctuation of c+ and c- in each half of
    the gap, in wall units of its own wall (y+ = distance from the wall times
    Re u_tau, u_tau from the mean wall shear of both walls), with the peak
    value; NaN before the first sample."""
    yc = np.asarray(st["yc"], dtype=np.float64)
    out = {}
    u_tau = st["u_tau"]
    for f in ("cp", "cm"):
        r = np.asarray(st["rms"][f], dtype=np.float64)
        for half, sel, dist in (("lower", yc < 0.0, yc + 1.0), ("upper", yc > 0.0, 1.0 - yc)):
            idx = np.flatnonzero(sel)
            if not len(idx) or not np.all(np.isfinite(r[idx])) or not (u_tau > 0):
                out[f"{f}_{half}"] = {"y_plus": float("nan"), "rms": float("nan")}
                continue
            m = idx[np.argmax(r[idx])]
            out[f"{f}_{half}"] = {"y_plus": float(dist[m] * cfg.re * u_tau), "rms": float(r[m])}
    return out


def main():
    ap = argparse.ArgumentParser(description="statistics campaign of one run (c_f, Re_tau, profiles)")
    ap.add_argument("--workload", default="couette_turbulent", choices=sorted(configs.WORKLOADS))
    ap.add_argument("--case", default=None, choices=sorted(TABLE1),
                    help="the paper's case parameters (Re, Sc, Debye length, beta); explicit flags override")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--vhat", type=float, default=0.0, help="wall potential difference in thermal volts")
    ap.add_argument("--debye", type=float, default=None)
    ap.add_argument("--sc", type=float, default=None)
    ap.add_argument("--re", type=float, default=None)
    ap.add_argument("--ny", type=int, default=None, help="wall-normal node count (resolution of the double layer)")
    ap.add_argument("--beta", type=float, default=None, help="electrokinetic coupling beta")
    ap.add_argument("--migration-face", type=int, default=0, choices=[0, 1, 2],
                    help="1: hybrid face value of the migration flux (upwind where |dPhi| >= 2); "
                         "2: also limited advective face values of the ions")
    ap.add_argument("--t-spin", type=float, default=150.0)
    ap.add_argument("--t-avg", type=float, default=200.0)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--amp", type=float, default=0.3)
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--ion-start", default="equilibrium", choices=["equilibrium", "uniform"],
                    help="ions from the zero-flow equilibrium double layer or uniform (c+- = 1)")
    ap.add_argument("--t-charge", type=float, default=None,
                    help="start uncharged and apply the wall voltage (with the equilibrium double layer) "
                         "at this time")
    ap.add_argument("--out", default="campaign_report.json")
    ap.add_argument("--metrics", default=None, help="append one JSON line of run metrics per monitor interval")
    ap.add_argument("--metrics-kernels", action="store_true",
                    help="include per-class kernel ms from the event profiler in the metrics lines")
    a = ap.parse_args()
    cfg = configs.WORKLOADS[a.workload](precision=a.precision)
    over = {"vhat": a.vhat, "u_noise": 0.0, "c_noise": 0.0, "migration_face": a.migration_face}
    if a.case:
        over.update(TABLE1[a.case])
    for k in ("debye", "sc", "re", "ny", "beta"):
        if getattr(a, k) is not None:
            over[k] = getattr(a, k)
    cfg = dataclasses.replace(cfg, **over)
    rep = run_campaign(cfg, a.t_spin, a.t_avg, every=a.every, amp=a.amp, ckpt=a.ckpt, resume=a.resume,
                       ion_start=a.ion_start, t_charge=a.t_charge,
                       log=lambda m: print(m, flush=True), metrics=a.metrics, metrics_kernels=a.metrics_kernels)
    Path(a.out).write_text(json.dumps(rep, indent=1) + "\n")
    if rep["stopped"]:
        print(f"[campaign] stopped early at t = {rep['stopped']['t']:.2f}: {rep['stopped']['reason']}", flush=True)
    print(f"[campaign] c_f = {rep['cf']:.4e} +- {rep['cf_stderr']:.1e}  Re_tau = {rep['re_tau']:.1f} "
          f"+- {rep['re_tau_stderr']:.1f}  (paper: c_f {PAPER_CF:.3e}, Re_tau {PAPER_RE_TAU:.0f}); "
          f"{rep['substeps']} substeps in {rep['wall_s']:.1f} s", flush=True)
    pk = rep["rms_peaks"]
    print("[campaign] RMS peaks (y+, rms): " + "  ".join(
        f"{k} ({v['y_plus']:.1f}, {v['rms']:.3e})" for k, v in pk.items()), flush=True)


if __name__ == "__main__":
    main()
