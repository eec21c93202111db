"""Pins of the hybrid face value of the migration flux (CPU only).

Sec. II discretises with second-order central differences: the face value of
c in the migration flux is the mean of the two cells.  Its stationary cell
ratio c_R / c_L = (1 - z dPhi/2) / (1 + z dPhi/2) is negative once the
potential difference across a face exceeds 2, which is where the paper's
large-voltage runs lose stability (Sec. III).  The hybrid rule (configuration
migration_face = 1) takes the upwind cell of the species' drift on those
faces and the mean elsewhere.  Pinned here:
  * the plane-averaged flux equals the upwind flux, computed by hand, on
    faces with |dPhi| >= 2 and the central flux on the others;
  * the explicit ion term is the divergence of that same flux (update and
    flux diagnostic use the same face values);
  * the zero-shear stationary state is positive where the central rule's is
    not, and satisfies the upwind zero-flux ratio 1/(1 + z dPhi) or
    1 + |dPhi| face by face;
  * ion mass is conserved to round-off and the wall flux is exactly zero in
    a sheared, noisy 3-D run with the rule active;
  * with the rule off, or with every |dPhi| < 2, results equal the central
    scheme bit for bit.
"""
import numpy as np
import pytest


@pytest.fixture(autouse=True)
def _few_threads(oracle_mod):
    oracle_mod.set_threads(2)
    yield
    oracle_mod.set_threads(8)


def _layer(oracle_mod, face, **kw):
    """Zero-shear 1-D cell column (nx = nz = 1), coarse in y so that the
    stationary double layer has potential jumps above 2 between cells."""
    args = dict(nx=1, ny=9, nz=1, re=1.0, sc=1.0, debye=0.1, vhat=20.0, u_top=0.0, u_bot=0.0, dt=2e-4,
                stretch=1.5, migration_face=face)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    return o


def _face_dphi(o):
    """Potential differences Phi_j - Phi_{j-1} across the interior y faces."""
    yc = o.yc
    Phi = 0.5 * o.cfg.vhat * yc + o.field("phi")[:, 0, 0]
    return np.diff(Phi)


def test_flux_is_upwind_on_steep_faces_and_central_elsewhere(oracle_mod):
    o = _layer(oracle_mod, 1)
    M = o.M
    rng = np.random.default_rng(1)
    cp = 1.0 + 0.4 * rng.uniform(size=M)
    cm = 1.0 + 0.4 * rng.uniform(size=M)
    phi = 3.0 * rng.standard_normal(M)
    o.field("cp")[:, 0, 0] = cp
    o.field("cm")[:, 0, 0] = cm
    o.field("phi")[:, 0, 0] = phi
    dphi = _face_dphi(o)
    steep = np.abs(dphi) >= 2.0
    assert steep.any() and (~steep).any()
    jp, jm, _, _ = o.ion_flux()
    kd = 1.0 / (o.cfg.re * o.cfg.sc)
    dc = o.dc[1:M]
    for c, z, j in ((cp, 1.0, jp), (cm, -1.0, jm)):
        cL, cR = c[:-1], c[1:]
        up = np.where(z * dphi > 0, cR, cL)
        cf = np.where(steep, up, 0.5 * (cL + cR))
        expect = -kd * ((cR - cL) / dc + z * cf * dphi / dc)
        np.testing.assert_allclose(j[1:M], expect, rtol=1e-12, atol=1e-14)
        assert j[0] == 0.0 and j[M] == 0.0


def test_explicit_term_is_the_divergence_of_the_flux(oracle_mod):
    """Quiescent 1-D state: the explicit ion term is the migration part only
    (wall-normal diffusion is implicit), and must equal minus the divergence
    of the plane-averaged migration flux over the cell heights."""
    o = _layer(oracle_mod, 1, ny=17)
    M = o.M
    rng = np.random.default_rng(2)
    o.field("cp")[:, 0, 0] = 1.0 + 0.5 * rng.uniform(size=M)
    o.field("cm")[:, 0, 0] = 1.0 + 0.5 * rng.uniform(size=M)
    o.field("phi")[:, 0, 0] = 2.5 * rng.standard_normal(M)
    o.field("u")[...] = 0.0
    o.field("v")[...] = 0.0
    o.field("w")[...] = 0.0
    assert (np.abs(_face_dphi(o)) >= 2.0).any()
    h = o.explicit_terms()
    jp, jm, _, _ = o.ion_flux()
    kd = 1.0 / (o.cfg.re * o.cfg.sc)
    dc, dn = o.dc, o.dn
    for name, j in (("cp", jp), ("cm", jm)):
        c = o.field(name)[:, 0, 0]
        jd = np.zeros(M + 1)
        jd[1:M] = -kd * np.diff(c) / dc[1:M]
        jmig = j - jd
        div = -(jmig[1:] - jmig[:-1]) / dn
        np.testing.assert_allclose(h[name][:, 0, 0], div, rtol=1e-11, atol=1e-12 * np.max(np.abs(div)))


def test_stationary_layer_is_positive_with_upwind_ratios(oracle_mod):
    """ny = 17, lam = 0.05, vhat = 40: the first two interior faces at each
    wall carry jumps of about 5.3 and 2.7, the rest stay below 2."""
    o = _layer(oracle_mod, 1, ny=17, debye=0.05, vhat=40.0, dt=0.0, cfl=0.5)
    while o.t < 6.0:  # many diffusion times of the gap at Re Sc = 1 (dt from the Debye limit)
        o.run(3000)
    cp = o.field("cp")[:, 0, 0].copy()
    cm = o.field("cm")[:, 0, 0].copy()
    assert np.all(cp > 0) and np.all(cm > 0)
    jp, jm, mp, mm = o.ion_flux()
    scale = max(cp.max(), cm.max()) / (o.cfg.re * o.cfg.sc * o.dc.min())  # natural flux scale
    assert np.max(np.abs(jp)) < 1e-11 * scale and np.max(np.abs(jm)) < 1e-11 * scale
    dphi = _face_dphi(o)
    steep = np.abs(dphi) >= 2.0
    assert steep.sum() >= 4 and (~steep).sum() >= 4
    for c, z in ((cp, 1.0), (cm, -1.0)):
        ratio = c[1:] / c[:-1]
        up = np.where(z * dphi > 0, 1.0 / (1.0 + z * dphi), 1.0 - z * dphi)
        central = (1 - z * dphi / 2) / (1 + z * dphi / 2)
        expect = np.where(steep, up, central)
        np.testing.assert_allclose(ratio, expect, rtol=1e-7)
        # on the steep faces the central rule's stationary ratio is negative
        assert np.all(central[steep] < 0)
    # counter-ions gather at the wall of opposite sign, symmetric layers
    assert cp[0] > 1 and cm[-1] > 1
    np.testing.assert_allclose(cp, cm[::-1], rtol=1e-9)


def test_central_rule_loses_positivity_on_the_same_grid(oracle_mod):
    o = _layer(oracle_mod, 0, ny=17, debye=0.05, vhat=40.0, dt=0.0, cfl=0.5)
    lowest = np.inf
    for _ in range(40):
        o.run(1500)
        c = np.concatenate([o.field("cp").ravel(), o.field("cm").ravel()])
        if not np.all(np.isfinite(c)):
            lowest = -np.inf
            break
        lowest = min(lowest, float(c.min()))
    assert lowest < 0


def test_mass_and_wall_flux_in_sheared_noisy_run(oracle_mod):
    """Coarse in y with vhat = 40: the applied field alone puts 5-6 thermal
    volts across most cell faces from the start."""
    o = oracle_mod.Oracle(nx=16, ny=9, nz=8, re=200.0, sc=1.0, debye=0.08, vhat=40.0, dt=0.0, cfl=0.4,
                          migration_face=1)
    o.init(5, 0.05, 1e-3)
    _, _, mp0, mm0 = o.ion_flux()
    steep_seen = False
    for _ in range(10):
        o.run(30)
        steep_seen |= bool(np.any(np.abs(np.diff(0.5 * o.cfg.vhat * o.yc[:, None, None] + o.field("phi"),
                                                 axis=0)) >= 2.0))
        jp, jm, mp, mm = o.ion_flux()
        assert jp[0] == 0.0 and jp[-1] == 0.0 and jm[0] == 0.0 and jm[-1] == 0.0
        assert abs(mp - mp0) < 1e-13 * mp0 and abs(mm - mm0) < 1e-13 * mm0
    assert steep_seen
    assert o.field("cp").min() > 0 and o.field("cm").min() > 0


def test_rule_is_inactive_below_the_threshold(oracle_mod):
    """Gentle layer (all jumps < 2): hybrid and central runs are identical."""
    runs = []
    for face in (0, 1):
        o = oracle_mod.Oracle(nx=8, ny=17, nz=4, re=100.0, debye=0.2, vhat=2.0, migration_face=face)
        o.init(3, 0.02, 1e-3)
        o.run(60)
        assert np.max(np.abs(_face_dphi_3d(o))) < 2.0
        runs.append(o.state())
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k


def _face_dphi_3d(o):
    Phi = 0.5 * o.cfg.vhat * o.yc[:, None, None] + o.field("phi")
    return np.concatenate([np.diff(Phi, axis=0).ravel(), np.diff(Phi, axis=1).ravel(),
                           np.diff(Phi, axis=2).ravel()])
