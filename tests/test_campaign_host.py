"""Host logic of the statistics campaign (no GPU): the batch-means error bar
of a correlated series."""
import math

import numpy as np

from paper_1701_02005_amd.campaign import batch_means


def test_batch_means_of_independent_samples():
    rng = np.random.default_rng(3)
    ses = []
    for _ in range(200):
        x = 2.0 + 0.5 * rng.standard_normal(1000)
        m, se = batch_means(x, 10)
        assert abs(m - x.mean()) < 1e-12
        ses.append(se)
    # standard error of the mean of 1000 iid samples of sd 0.5
    assert abs(np.mean(ses) / (0.5 / math.sqrt(1000)) - 1.0) < 0.1


def test_batch_means_sees_correlation():
    """An AR(1) series with correlation time ~50 samples: batch means over
    batches of 1000 give the larger, correct standard error."""
    rng = np.random.default_rng(5)
    phi, n = 0.98, 20000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    _, se = batch_means(x, 20)
    naive = x.std() / math.sqrt(n)
    exact = math.sqrt(1 / (1 - phi ** 2)) * math.sqrt((1 + phi) / (1 - phi)) / math.sqrt(n)
    assert se > 3 * naive
    assert 0.5 < se / exact < 1.6


def test_equilibrium_double_layer_is_stationary_in_the_oracle(oracle_mod):
    """The campaign's zero-flow equilibrium double layer, computed on the
    host from the discrete zero-flux condition, is left unchanged by the
    oracle's substeps without shear (ion transport, potential, Coulomb force
    and pressure all in balance), is mirror-symmetric, and is uniform without
    voltage."""
    import dataclasses
    import paper_1701_02005_amd as P
    from paper_1701_02005_amd.campaign import equilibrium_ions
    cfg = dataclasses.replace(P.configs.couette_small(), nx=4, nz=4, ny=33, vhat=4.0, debye=1 / 33, sc=3.0,
                              re=1.0, u_top=0.0, u_bot=0.0, u_noise=0.0, c_noise=0.0, dt=2e-4)
    cp, cm, phi = equilibrium_ions(cfg)
    assert abs(np.sum(cp * np.diff(P.grid(cfg)[0])) - 2.0) < 1e-12
    assert np.max(np.abs(cp - cm[::-1])) < 1e-10 * cp.max() and cp[0] > 3 and cp[-1] < 0.3
    oracle_mod.set_threads(1)
    o = oracle_mod.Oracle(**cfg.oracle_kwargs())
    o.init(0, 0.0, 0.0)
    o.field("cp")[...] = cp[:, None, None]
    o.field("cm")[...] = cm[:, None, None]
    o.solve_potential()
    assert np.max(np.abs(o.field("phi")[:, 0, 0] - phi)) < 1e-10 * np.max(np.abs(phi))
    o.run(30)
    assert np.max(np.abs(o.field("cp")[:, 0, 0] - cp)) < 1e-10 * cp.max()
    assert np.max(np.abs(o.field("cm")[:, 0, 0] - cm)) < 1e-10 * cm.max()
    oracle_mod.set_threads(8)
    cp0, cm0, phi0 = equilibrium_ions(dataclasses.replace(cfg, vhat=0.0))
    assert np.max(np.abs(cp0 - 1.0)) < 1e-14 and np.max(np.abs(phi0)) < 1e-14


def test_rms_peaks_in_wall_units():
    """Peak of a synthetic RMS profile, one per half: y+ is the distance of
    the peak row from its own wall times Re u_tau."""
    from types import SimpleNamespace
    from paper_1701_02005_amd.campaign import rms_peaks
    yc = np.linspace(-0.95, 0.95, 20)
    r_cp = np.exp(-((yc + 0.85) / 0.05) ** 2) + 0.5 * np.exp(-((yc - 0.75) / 0.05) ** 2)
    r_cm = np.exp(-((yc + 0.65) / 0.05) ** 2) + 2.0 * np.exp(-((yc - 0.95) / 0.05) ** 2)
    st = {"yc": yc, "rms": {"cp": r_cp, "cm": r_cm}, "u_tau": 0.05}
    pk = rms_peaks(st, SimpleNamespace(re=3000.0))
    scale = 3000.0 * 0.05
    assert abs(pk["cp_lower"]["y_plus"] - (yc[1] + 1) * scale) < 1e-9
    assert abs(pk["cp_upper"]["y_plus"] - (1 - yc[17]) * scale) < 1e-9
    assert abs(pk["cm_lower"]["y_plus"] - (yc[3] + 1) * scale) < 1e-9
    assert abs(pk["cm_upper"]["y_plus"] - (1 - yc[19]) * scale) < 1e-9
    assert pk["cm_upper"]["rms"] == r_cm[19]
    st["u_tau"] = float("nan")
    assert np.isnan(rms_peaks(st, SimpleNamespace(re=3000.0))["cp_lower"]["y_plus"])


def test_metrics_record_from_a_stub_solver():
    """The metrics line's derived values: c_f = 2 tau and Re_tau = Re
    sqrt(tau) from the mean wall stress, the KE-budget residual between two
    records, and per-launch kernel times from the profiler's running totals."""
    from types import SimpleNamespace
    from paper_1701_02005_amd.campaign import metrics_record

    class Stub:
        def __init__(self, t, ke, ww, dis, fw, prof):
            self.cfg = SimpleNamespace(re=400.0)
            self._t, self._ke, self._e, self._prof = t, ke, (ww, dis, fw), prof

        def clock(self):
            return self._t, 1e-3, 0, int(self._t * 1000)

        def wall_shear_stress(self):
            return 2.4e-3, 2.6e-3

        def ion_flux(self):
            return [0.0], [0.0], 4.0, 4.0

        def diagnostics(self):
            return {"ke": self._ke, "max_div": 1e-14, "min_cp": 0.9, "min_cm": 0.8, "max_dphi": 0.5}

        def energy_budget(self):
            return dict(zip(("wall_work", "dissipation", "force_work"), self._e))

        def profile_read(self):
            return self._prof

    a = metrics_record(Stub(1.0, 1.0, 0.30, 0.10, 0.0, {"explicit_rhs": (4.0, 2)}), None, kernels=True)
    assert abs(a["cf"] - 5.0e-3) < 1e-15 and abs(a["re_tau"] - 400.0 * math.sqrt(2.5e-3)) < 1e-12
    assert "budget_residual" not in a and a["kernel_ms"] == {"explicit_rhs": 2.0}
    b = metrics_record(Stub(1.5, 1.1, 0.30, 0.10, 0.0, {"explicit_rhs": (10.0, 5)}), a, kernels=True)
    assert abs(b["budget_residual"] - (0.2 - 0.2)) < 1e-12  # dKE/dt = 0.2 = wall work - dissipation
    assert abs(b["kernel_ms"]["explicit_rhs"] - 2.0) < 1e-12  # (10 - 4) ms over 3 launches
    c = metrics_record(Stub(2.0, 1.1, 0.30, 0.10, -0.05, {}), b)
    assert abs(c["budget_residual"] - (0.0 - 0.175)) < 1e-12
