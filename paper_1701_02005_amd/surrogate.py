"""Learned warm start for new runs.

Pipeline (all GPU work through the HIP library):

1. an ensemble of independent runs over (Re, vhat, Debye length) is advanced
   together, long enough for the double layer of every run to become
   stationary; each run's lower-half charge is recorded chunk by chunk and
   the stationarity rule below decides which runs are stationary over the
   averaging window (only those are training data);
2. the time-mean plane profiles of u, rho = c+ - c- and Phi over the
   averaging window are sampled at each run's wall-normal nodes (wall values
   from the boundary conditions: u = u_bot / u_top, Phi = -+vhat/2, rho
   linearly extrapolated) and interpolated onto the nodes of the target grid;
3. a GELU network (BF16 matrix-core kernels, Adam) learns the map from the
   scaled control parameters to the encoded profiles (u as is, asinh(rho),
   Phi / (vhat/2 + 1e-6), each standardised);
4. new runs are initialised from its predictions: u = predicted mean profile
   plus the same seeded noise as the plain start, c+- rebuilt from rho with
   c+ c- = A^2 and both ion contents fixed, phi re-solved;
5. warm and plain starts are advanced side by side and the times after which
   the mean wall shear stress and the charge of the lower half gap (the
   quantity the double layer sets) stay within 1 % of their stationary
   values are compared.

The stationarity rule: the reference is the mean over the second half of
the plain run; t* is the first time after which the average over a window
of `window` time units stays within `tol` of the reference to the end of
the run (censored at the end when it never does).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import re as regex
import time
from pathlib import Path

import numpy as np

from . import configs
from .binding import Config, Ensemble, Mlp, NsPnpError, grid

SIZES = (3, 256, 256, 256, 256, 579)
RANGES = {"re": (500.0, 3000.0), "vhat": (0.0, 20.0), "lnlam": (math.log(0.02), math.log(0.2))}


# ---------------------------------------------------------------- features
def scale_inputs(re, vhat, lam, ranges=RANGES) -> np.ndarray:
    """(Re, vhat, ln lam) mapped linearly onto [-1, 1] over the sampling ranges."""
    cols = []
    for val, key in ((np.asarray(re, float), "re"), (np.asarray(vhat, float), "vhat"),
                     (np.log(np.asarray(lam, float)), "lnlam")):
        lo, hi = ranges[key]
        cols.append(2.0 * (val - lo) / (hi - lo) - 1.0)
    return np.stack(cols, axis=-1)


def sample_points(seed: int, n: int, ranges=RANGES):
    """Point i: (Re, vhat, lam) from a generator seeded with (seed, i): Re and
    vhat uniform, lam log-uniform over the ranges (the ensemble sampler)."""
    pts = []
    for i in range(n):
        rng = np.random.default_rng([seed, i])
        re = float(rng.uniform(*ranges["re"]))
        vhat = float(rng.uniform(*ranges["vhat"]))
        lam = float(math.exp(rng.uniform(*ranges["lnlam"])))
        pts.append((re, vhat, lam))
    return pts


def node_profiles(cfg: Config, u_c, rho_c, phi_c):
    """Cell-row means -> node values including the walls (see module doc)."""
    yn, yc = (np.asarray(a) for a in grid(cfg))
    u_c, rho_c, phi_c = (np.asarray(a, float) for a in (u_c, rho_c, phi_c))
    Phi_c = 0.5 * cfg.vhat * yc + phi_c
    inner = yn[1:-1]
    u = np.concatenate([[cfg.u_bot], np.interp(inner, yc, u_c), [cfg.u_top]])
    Phi = np.concatenate([[-0.5 * cfg.vhat], np.interp(inner, yc, Phi_c), [0.5 * cfg.vhat]])
    r0 = rho_c[0] + (rho_c[1] - rho_c[0]) * (yn[0] - yc[0]) / (yc[1] - yc[0])
    r1 = rho_c[-1] + (rho_c[-1] - rho_c[-2]) * (yn[-1] - yc[-1]) / (yc[-1] - yc[-2])
    rho = np.concatenate([[r0], np.interp(inner, yc, rho_c), [r1]])
    return yn, u, rho, Phi


def encode(u, rho, Phi, vhat) -> np.ndarray:
    return np.concatenate([u, np.arcsinh(rho), Phi / (0.5 * vhat + 1e-6)])


def decode(vec, vhat, n):
    u = vec[:n]
    rho = np.sinh(vec[n:2 * n])
    Phi = vec[2 * n:3 * n] * (0.5 * vhat + 1e-6)
    return u, rho, Phi


@dataclasses.dataclass
class Standardizer:
    mean: np.ndarray
    std: np.ndarray

    @classmethod
    def fit(cls, Y):
        return cls(Y.mean(axis=0), np.maximum(Y.std(axis=0), 1e-6))

    def fwd(self, Y):
        return (Y - self.mean) / self.std

    def inv(self, Z):
        return Z * self.std + self.mean


def ions_from_charge(rho_c, dn, info: dict | None = None):
    """c+- = (sqrt(rho^2 + 4 A^2) +- rho) / 2 (Boltzmann product c+ c- = A^2),
    rho shifted to zero net charge, A fixed so that sum(c+- dy) = 2.  A
    charge the ions cannot carry (sum |rho| dy at or above the total content,
    where no A > 0 exists and one species would be zero) is first scaled to
    99% of it; info, if given, receives that factor.  The minority species is
    formed as A^2 / c_majority (no cancellation)."""
    rho = np.asarray(rho_c, float)
    dn = np.asarray(dn, float)
    rho = rho - np.sum(rho * dn) / np.sum(dn)
    target = 2.0 * np.sum(dn)  # sum(c+ + c-) dy = 4 over the gap of 2
    mag = np.sum(np.abs(rho) * dn)
    scale = 1.0 if mag < 0.99 * target else 0.99 * target / mag
    rho = rho * scale
    if info is not None:
        info["scale"] = scale

    def total(A):
        return np.sum(np.sqrt(rho * rho + 4 * A * A) * dn)

    lo, hi = 0.0, 1.0
    while total(hi) < target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    A = 0.5 * (lo + hi)
    big = 0.5 * (np.sqrt(rho * rho + 4 * A * A) + np.abs(rho))
    small = A * A / big
    return np.where(rho >= 0, big, small), np.where(rho >= 0, small, big), A


def stationary_time(t, series, ref, window, tol):
    """First time after which the trailing-window average stays within tol*|ref|."""
    t = np.asarray(t, float)
    s = np.asarray(series, float)
    ok = np.zeros(len(t), bool)
    for q in range(len(t)):
        sel = (t > t[q] - window) & (t <= t[q])
        avg = s[sel].mean()
        ok[q] = abs(avg - ref) <= tol * abs(ref) and t[q] - t[0] >= min(window, t[-1] - t[0])
    bad = np.nonzero(~ok)[0]
    if len(bad) == 0:
        return float(t[0]), False
    last_bad = bad[-1]
    if last_bad == len(t) - 1:
        return float(t[-1]), True  # censored
    return float(t[last_bad + 1]), False


def lower_half_charge(cfg: Config, rho):
    """Charge of the lower half gap per unit wall area, sum over the rows
    below the mid-plane of rho dy."""
    yn, yc = (np.asarray(a) for a in grid(cfg))
    low = yc < 0
    return float(np.sum(np.asarray(rho)[low] * np.diff(yn)[low]))


# ---------------------------------------------------------------- stages
def ensemble_data(members, substeps: int, window_substeps: int, target: Config, chunk: int = 3000,
                  tol: float = 0.01, log=print, tune_cache=None):
    """Advance the training ensemble substeps substeps in graph replays of
    chunk substeps; per chunk, every run's chunk-mean profiles.  A run is
    training data when its lower-half charge, chunk by chunk, stays within
    tol of its mean over the last window_substeps throughout that window.
    Returns inputs X, encoded targets Y (runs kept), target nodes, report."""
    t0 = time.perf_counter()
    ens = Ensemble(members)
    tiles = ens.autotune(tune_cache, 6)
    done = ens.clock(0)[2]
    ens.stats(True)      # on before the capture: the replayed graph then includes the statistics kernel
    ens.capture(chunk)
    nchunk = max(1, (substeps - done) // chunk)
    series = [[] for _ in members]  # (t, q, wt, u, rho, phi) per chunk
    for it in range(nchunk):
        ens.stats(True)
        ens.step(chunk)
        for m, c in enumerate(members):
            u, rho, phi, wt = ens.profiles(m)
            series[m].append((ens.clock(m)[0], lower_half_charge(c, rho), wt, u, rho, phi))
        if (it + 1) % 10 == 0 or it == nchunk - 1:
            log(f"ensemble: {done + chunk * (it + 1)} substeps, {time.perf_counter() - t0:.1f} s")
    ens.sync()
    wall = time.perf_counter() - t0
    y_t, _ = grid(target)
    nwin = max(1, window_substeps // chunk)
    X, Y, meta = [], [], []
    for m, c in enumerate(members):
        ser = series[m][-nwin:]
        wts = np.array([s[2] for s in ser])
        qs = np.array([s[1] for s in ser])
        qref = float(np.sum(wts * qs) / wts.sum())
        drift = float(np.max(np.abs(qs - qref)) / max(abs(qref), 1e-12))
        stationary = drift <= tol
        prof = [np.sum([w * np.asarray(s[k]) for w, s in zip(wts, ser)], axis=0) / wts.sum() for k in (3, 4, 5)]
        try:
            dg = ens.diagnostics(m)
        except Exception as exc:  # non-finite member
            dg = {"error": str(exc)}
            stationary = False
        meta.append({"re": c.re, "vhat": c.vhat, "debye": c.debye, "grid": f"{c.nx}x{c.ny}x{c.nz}",
                     "t_end": series[m][-1][0], "window_start_t": ser[0][0] - 0.0, "charge": qref,
                     "charge_drift": drift, "stationary": stationary, "diagnostics": dg})
        if stationary:
            yn, u, rho, Phi = node_profiles(c, *prof)
            ui, ri, Pi = (np.interp(y_t, yn, f) for f in (u, rho, Phi))
            X.append((c.re, c.vhat, c.debye))
            Y.append(encode(ui, ri, Pi, c.vhat))
    points = sum(c.points for c in members) * substeps
    kept = len(X)
    log(f"ensemble: {len(members)} runs, {substeps} substeps in {wall:.1f} s "
        f"({points / wall / 1e6:.0f} Mpoint-substeps/s incl. autotune and capture); "
        f"{kept} stationary in charge over the last {nwin} chunks; member times "
        f"{min(r['t_end'] for r in meta):.1f} .. {max(r['t_end'] for r in meta):.1f}")
    info = {"members": len(members), "substeps": substeps, "window_substeps": nwin * chunk, "chunk": chunk,
            "tol": tol, "wall_s": wall, "mpoint_substeps_per_s": points / wall / 1e6, "tiles": tiles,
            "stationary": kept, "runs": meta}
    return np.array(X), np.array(Y), np.asarray(y_t), info


def init_params(sizes, seed):
    """He-style uniform initialisation (W [in, out], zero biases), flattened."""
    rng = np.random.default_rng(seed)
    out = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        b = math.sqrt(6.0 / fin)
        out.append(rng.uniform(-b, b, (fin, fout)).ravel())
        out.append(np.zeros(fout))
    return np.concatenate(out).astype(np.float32)


def train_network(X, Y, steps: int, lr: float, seed: int, sizes=SIZES, ranges=RANGES, log=print):
    import torch
    xs = scale_inputs(X[:, 0], X[:, 1], X[:, 2], ranges).astype(np.float32)
    std = Standardizer.fit(Y)
    ys = std.fwd(Y).astype(np.float32)
    net = Mlp(sizes, max(64, len(xs)), init_params(sizes, seed))
    xt = torch.tensor(xs, device=net.device)
    yt = torch.tensor(ys, device=net.device)
    losses = []
    t0 = time.perf_counter()
    for it in range(steps):
        lt = net.train_step(xt, yt, lr)
        if it % 250 == 0 or it == steps - 1:
            losses.append((it, float(lt.item())))
    net.sync()
    wall = time.perf_counter() - t0
    final = net.gradients(xt, yt)
    log(f"training: {steps} Adam steps in {wall:.2f} s, loss {losses[0][1]:.3e} -> {final:.3e}")
    return net, std, {"steps": steps, "lr": lr, "wall_s": wall, "loss_curve": losses, "final_loss": final,
                      "samples": int(len(xs))}


def predict(net, std, X, ranges=RANGES):
    import torch
    xs = torch.tensor(scale_inputs(X[:, 0], X[:, 1], X[:, 2], ranges).astype(np.float32), device=net.device)
    out = net.forward(xs).cpu().numpy().astype(np.float64)
    return std.inv(out)


def test_members(seed: int, n: int, base: Config, ranges=RANGES):
    """Unseen parameter points (the sampler with another seed) on the grid of base."""
    return [dataclasses.replace(base, re=re, vhat=vhat, debye=lam, seed=base.seed + 7 * q)
            for q, (re, vhat, lam) in enumerate(sample_points(seed, n, ranges))]


def warm_start(ens: Ensemble, members, preds, y_t, log=print):
    import torch
    for m, (c, vec) in enumerate(zip(members, preds)):
        u_t, rho_t, Phi_t = decode(vec, c.vhat, len(y_t))
        yn, yc = (np.asarray(a) for a in grid(c))
        dn = np.diff(yn)
        u_new = np.interp(yc, y_t, u_t)
        u_lin = 0.5 * (c.u_top + c.u_bot) + 0.5 * (c.u_top - c.u_bot) * yc
        info = {}
        cp_new, cm_new, _ = ions_from_charge(np.interp(yc, y_t, rho_t), dn, info)
        if info["scale"] < 1.0:
            log(f"warm start {m}: predicted charge beyond the ion content, scaled by {info['scale']:.3f}")
        shape = (c.ny - 1, c.nz, c.nx)
        u = ens.get_field(m, "u") + torch.tensor(u_new - u_lin, device=ens.device).view(-1, 1, 1)
        # the plain start's seeded ion noise (1 + n, |n| <= c_noise) carried as a
        # relative factor: added as it stands it would exceed the co-ion
        # concentration of a strong double layer near the walls (4e-5 at
        # vhat 19, lam 0.028) and start the run negative; each content is
        # rescaled to its noise-free value
        dv = torch.tensor(dn, device=ens.device).view(-1, 1, 1)

        def with_noise(name, prof):
            base = torch.tensor(prof, device=ens.device).view(-1, 1, 1)
            val = ens.get_field(m, name) * base
            return val * ((base * dv).sum() * c.nx * c.nz / (val * dv).sum())

        cp, cm = with_noise("cp", cp_new), with_noise("cm", cm_new)
        for name, val in (("u", u), ("cp", cp), ("cm", cm)):
            ens.set_field(m, name, val.reshape(shape).contiguous())
        ens.refresh_potential(m)
    ens.sync()


def monitor(ens: Ensemble, members, chunk: int, t_end: float, log=print, max_substeps: int | None = None,
            label: str = ""):
    """Advance until every member reaches t_end (or max_substeps per member
    have run); per chunk record the chunk-mean wall shear stress and
    lower-half charge of every member.  Logs progress every 30 s."""
    out = [{"t": [], "tau": [], "q": []} for _ in members]
    geo = [tuple(np.asarray(a) for a in grid(c)) for c in members]
    t0 = time.perf_counter()
    t_log = t0
    nsub = 0
    while True:
        ens.stats(True)
        ens.step(chunk)
        nsub += chunk
        tmin = math.inf
        for m, c in enumerate(members):
            u, rho, phi, wt = ens.profiles(m)
            yn, yc = geo[m]
            t = ens.clock(m)[0]
            tb = (u[0] - c.u_bot) / (c.re * (yc[0] - yn[0]))
            tt = (c.u_top - u[-1]) / (c.re * (yn[-1] - yc[-1]))
            out[m]["t"].append(t)
            out[m]["tau"].append(0.5 * (tb + tt))
            out[m]["q"].append(lower_half_charge(c, rho))
            out[m].setdefault("prof", []).append((wt, u, rho, phi))
            tmin = min(tmin, t)
        now = time.perf_counter()
        if now - t_log >= 30.0:
            t_log = now
            log(f"{label}: {nsub} substeps, slowest member at t = {tmin:.1f}, {now - t0:.0f} s")
        if tmin >= t_end or (max_substeps is not None and nsub >= max_substeps):
            break
    ens.sync()
    wall = time.perf_counter() - t0
    return out, nsub, wall


def compare_starts(members, preds, y_t, t_end: float, chunk: int, window: float, tol: float, log=print,
                   max_substeps: int | None = None):
    """Plain and warm starts of the test runs advanced side by side; t* of
    the drag and of the lower-half charge for both, against the plain run's
    second-half mean.  max_substeps caps each start (the runs then end
    before t_end, which the report states per member)."""
    results, failed, start_diag = {}, {"plain": {}, "warm": {}}, {}
    for label in ("plain", "warm"):
        # a start that the health check stops (a negative concentration) is
        # recorded with its time and dropped; the others start again
        active = list(range(len(members)))
        while True:
            ens = Ensemble([members[i] for i in active])
            init_s = 0.0
            if label == "warm":
                t0 = time.perf_counter()
                warm_start(ens, [members[i] for i in active], [preds[i] for i in active], y_t, log)
                init_s = time.perf_counter() - t0
                for q, i in enumerate(active):
                    try:
                        start_diag.setdefault(i, ens.diagnostics(q))
                    except NsPnpError as exc:
                        start_diag.setdefault(i, {"error": str(exc)})
            ens.stats(True)  # on before the capture (the graph then includes the statistics kernel)
            ens.capture(chunk)
            try:
                series, nsub, wall = monitor(ens, [members[i] for i in active], chunk, t_end, log, max_substeps,
                                             label)
            except NsPnpError as exc:
                hit = regex.search(r"ensemble member (\d+)", str(exc))
                if hit is None:
                    raise
                i = active[int(hit.group(1))]
                try:
                    t_fail = ens.clock(int(hit.group(1)))[0]
                except NsPnpError:
                    t_fail = float("nan")
                failed[label][i] = {"t": t_fail, "reason": str(exc)}
                log(f"{label}: run {i} stopped at t = {t_fail:.2f} ({exc}); continuing without it")
                active.remove(i)
                del ens
                if not active:
                    series, nsub, wall = [], 0, 0.0
                    break
                continue
            break
        results[label] = (dict(zip(active, series)), nsub, wall, init_s)
        log(f"{label}: {nsub} substeps per run to t >= {t_end} in {wall:.1f} s")
        del ens
    plain, _, wall_p, _ = results["plain"]
    warm, _, wall_w, init_w = results["warm"]
    per = []
    for m, c in enumerate(members):
        if m not in plain or m not in warm:
            rec = {"re": c.re, "vhat": c.vhat, "debye": c.debye, "failed_plain": failed["plain"].get(m),
                   "failed_warm": failed["warm"].get(m), "warm_start_state": start_diag.get(m)}
            per.append(rec)
            log(f"point {m}: Re={c.re:.0f} vhat={c.vhat:.2f} lam={c.debye:.4f}  stopped: "
                f"plain {failed['plain'].get(m, {}).get('t')} warm {failed['warm'].get(m, {}).get('t')} "
                f"(warm start min c {start_diag.get(m, {}).get('min_cm', float('nan')):.3e}, "
                f"max dPhi {start_diag.get(m, {}).get('max_dphi', float('nan')):.2f})")
            continue
        ps, ws = plain[m], warm[m]
        tp = np.array(ps["t"])
        half = tp >= 0.5 * tp[-1]
        rec = {"re": c.re, "vhat": c.vhat, "debye": c.debye, "warm_start_state": start_diag.get(m),
               "t_reached_plain": float(tp[-1]),
               "t_reached_warm": float(ws["t"][-1]), "capped": bool(tp[-1] < t_end or ws["t"][-1] < t_end)}
        for key in ("tau", "q"):
            ref = float(np.mean(np.array(ps[key])[half]))
            t_p, cen_p = stationary_time(ps["t"], ps[key], ref, window, tol)
            t_w, cen_w = stationary_time(ws["t"], ws[key], ref, window, tol)
            n_p = int(np.searchsorted(tp, t_p)) * chunk
            n_w = int(np.searchsorted(np.array(ws["t"]), t_w)) * chunk
            rec[key] = {"ref": ref, "t_plain": t_p, "t_warm": t_w, "censored_plain": cen_p, "censored_warm": cen_w,
                        "substeps_plain": n_p, "substeps_warm": n_w,
                        "wall_plain_s": wall_p * n_p / max(1, len(tp) * chunk),
                        "wall_warm_s": wall_w * n_w / max(1, len(ws["t"]) * chunk) + init_w}
        # profile error of the prediction against the plain run's late-time mean
        late = [p for p, h in zip(ps["prof"], half) if h]
        wts = np.array([p[0] for p in late])
        prof = [np.sum([w * np.asarray(p[i]) for w, p in zip(wts, late)], axis=0) / wts.sum() for i in (1, 2, 3)]
        yn, u, rho, Phi = node_profiles(c, *prof)
        truth = [np.interp(y_t, yn, f) for f in (u, rho, Phi)]
        pu, pr, pP = decode(preds[m], c.vhat, len(y_t))
        rec["profile_rel_l2"] = {k: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
                                 for k, a, b in (("u", pu, truth[0]), ("rho", pr, truth[1]), ("Phi", pP, truth[2]))}
        per.append(rec)
        log(f"point {m}: Re={c.re:.0f} vhat={c.vhat:.2f} lam={c.debye:.4f}  "
            f"drag t*: plain {rec['tau']['t_plain']:.2f} warm {rec['tau']['t_warm']:.2f} | "
            f"charge t*: plain {rec['q']['t_plain']:.2f}{'(c)' if rec['q']['censored_plain'] else ''} "
            f"warm {rec['q']['t_warm']:.2f}{'(c)' if rec['q']['censored_warm'] else ''} | "
            f"L2 u {rec['profile_rel_l2']['u']:.2e} rho {rec['profile_rel_l2']['rho']:.2e} "
            f"Phi {rec['profile_rel_l2']['Phi']:.2e}")
    return per, {"wall_plain_s": wall_p, "wall_warm_s": wall_w, "warm_init_s": init_w}


def run(out_path: str, seed: int = 0, ens_substeps: int = 240000, window_substeps: int = 30000,
        train_steps: int = 3000, lr: float = 1e-3, n_test: int = 8, test_plane: int = 32, t_end: float = 3000.0,
        chunk: int = 300, window: float = 5.0, tol: float = 0.01, precision: str = "mixed", log=print,
        max_substeps: int | None = None):
    """The experiment at the production sizes: the 64-run ensemble (hybrid
    migration face value, so that every voltage of the sampler stays
    positive) as training data, the 3 -> 4 x 256 -> 3 x 193 network, and
    n_test unseen points on the 193-node wall-normal grid of the turbulent
    workload with test_plane x test_plane horizontal points."""
    report = {"seed": seed}
    members = [dataclasses.replace(c, migration_face=1) for c in configs.ensemble_members(seed, precision=precision)]
    target = configs.couette_turbulent(precision=precision)
    X, Y, y_t, report["ensemble"] = ensemble_data(members, ens_substeps, window_substeps, target, log=log)
    net, std, report["training"] = train_network(X, Y, train_steps, lr, seed, log=log)
    # test runs with limited advective face values as well: the warm start
    # sets steep double layers and the start's velocity noise together, which
    # central advection can drive negative
    base = dataclasses.replace(target, nx=test_plane, nz=test_plane, migration_face=2)
    tests = test_members(seed + 1, n_test, base)
    Xt = np.array([(c.re, c.vhat, c.debye) for c in tests])
    t0 = time.perf_counter()
    preds = predict(net, std, Xt)
    report["inference_s"] = time.perf_counter() - t0
    log(f"test points: {[(round(c.re), round(c.vhat, 2), round(c.debye, 4)) for c in tests]}")
    per, walls = compare_starts(tests, preds, y_t, t_end, chunk, window, tol, log, max_substeps)
    report["test"] = {"points": per, "grid": f"{base.nx}x{base.ny}x{base.nz}", "t_end": t_end, "window": window,
                      "tol": tol, "chunk": chunk, **walls}
    Path(out_path).parent.mkdir(parents=True, exist_ok=True)
    Path(out_path).write_text(json.dumps(report, indent=1, default=float))
    return report


def main():
    ap = argparse.ArgumentParser(description="ensemble -> surrogate network -> warm-started runs")
    ap.add_argument("--out", default="surrogate_report.json")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ens-substeps", type=int, default=240000)
    ap.add_argument("--window-substeps", type=int, default=30000)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--n-test", type=int, default=8)
    ap.add_argument("--test-plane", type=int, default=32)
    ap.add_argument("--t-end", type=float, default=3000.0)
    ap.add_argument("--max-substeps", type=int, default=None, help="cap per start of the test runs")
    args = ap.parse_args()
    run(args.out, seed=args.seed, ens_substeps=args.ens_substeps, window_substeps=args.window_substeps,
        train_steps=args.train_steps, n_test=args.n_test, test_plane=args.test_plane, t_end=args.t_end,
        max_substeps=args.max_substeps,
        log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
