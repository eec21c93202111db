"""Physics pins of the oracle's whole time step (CPU only).

Closed forms, conservation laws and invariants that the discrete NS-PNP
scheme of Sec. II must reproduce:
  * laminar Couette flow is a steady state with wall stress 1/Re (Sec. II,
    definition of tau_w);
  * the projection leaves a discretely divergence-free field (Eq. (2));
  * ion mass is conserved and the wall-normal ion flux is zero on the walls
    (Fig. 1 caption);
  * the zero-shear stationary state is the Poisson-Boltzmann double layer
    (Sec. II), with the Debye-Hueckel profile at small voltage and symmetric
    profiles (Sec. II, electrokinetic validation);
  * hydrostatic balance of the Coulomb force: p - K (c+ + c-) is uniform
    (osmotic pressure), which fixes the coupling K and the force sign;
  * time accuracy: third order for the explicit Runge-Kutta part, second
    order for the Crank-Nicolson wall-normal diffusion;
  * the discrete kinetic-energy budget closes as dt -> 0;
  * the plane-Couette pi-rotation symmetry is preserved.
"""
import numpy as np
import pytest
from scipy.integrate import solve_bvp
from scipy.optimize import fsolve


@pytest.fixture(autouse=True)
def _few_threads(oracle_mod):
    oracle_mod.set_threads(1)
    yield
    oracle_mod.set_threads(8)


def _quiet(oracle_mod, **kw):
    args = dict(nx=1, ny=33, nz=1, re=1.0, sc=1.0, debye=0.1, vhat=5.0, u_top=0.0, u_bot=0.0,
                dt=5e-4, stretch=1.5)
    args.update(kw)
    o = oracle_mod.Oracle(**args)
    o.init(0, 0.0, 0.0)
    return o


# --------------------------------------------------------------------------
# laminar Couette flow
# --------------------------------------------------------------------------

def test_couette_is_exact_steady_state(oracle_mod):
    o = oracle_mod.Oracle(nx=16, ny=33, nz=8, vhat=0.0, re=400.0)
    o.init(0, 0.0, 0.0)
    yc = o.yc
    assert np.max(np.abs(o.field("u") - yc[:, None, None])) < 1e-15
    o.run(30)
    assert np.max(np.abs(o.field("u") - yc[:, None, None])) < 1e-14
    assert np.max(np.abs(o.field("v"))) < 1e-14 and np.max(np.abs(o.field("w"))) < 1e-14
    tb, tt = o.wall_shear()
    assert tb == pytest.approx(1 / 400.0, rel=1e-12) and tt == pytest.approx(1 / 400.0, rel=1e-12)


def test_couette_with_moving_walls_and_offset(oracle_mod):
    """Walls at (u_bot, u_top) = (-0.4, 1.6): u = 0.6 + y, tau = 1/Re."""
    o = oracle_mod.Oracle(nx=8, ny=17, nz=4, vhat=0.0, re=50.0, u_top=1.6, u_bot=-0.4)
    o.init(0, 0.0, 0.0)
    o.run(9)
    assert np.max(np.abs(o.field("u") - (0.6 + o.yc)[:, None, None])) < 1e-14
    tb, tt = o.wall_shear()
    assert tb == pytest.approx(1 / 50.0, rel=1e-12) and tt == pytest.approx(1 / 50.0, rel=1e-12)


# --------------------------------------------------------------------------
# divergence and conservation on the small production case
# --------------------------------------------------------------------------

def test_divergence_free_and_ion_mass_conserved(oracle_mod):
    oracle_mod.set_threads(8)
    o = oracle_mod.Oracle()  # 32x33x32, Re 400, lam 0.1, vhat 5, dt 1e-3
    o.init(0)
    _, _, mp0, mm0 = o.ion_flux()
    vol = 2.0 * o.cfg.lx * o.cfg.lz
    assert mp0 == pytest.approx(vol, rel=1e-14) and mm0 == pytest.approx(vol, rel=1e-14)
    assert o.max_divergence() < 1e-12
    for _ in range(10):
        o.run(20)
        assert o.max_divergence() < 1e-12
    jp, jm, mp, mm = o.ion_flux()
    assert abs(mp - mp0) / mp0 < 1e-13 and abs(mm - mm0) / mm0 < 1e-13
    assert jp[0] == 0.0 and jp[-1] == 0.0 and jm[0] == 0.0 and jm[-1] == 0.0
    assert o.t == pytest.approx(66e-3 + (8 / 15 + 2 / 15) * 1e-3, rel=1e-12)


# --------------------------------------------------------------------------
# zero-shear double layer
# --------------------------------------------------------------------------

def _discrete_pb(yn, yc, dn, dc, vhat, lam):
    """Stationary discrete PNP: zero total flux through every interior face,
    ion mass fixed, discrete Poisson with phi = 0 at the walls.  Written from
    the steady-state conditions, not from the time stepper."""
    M = len(yc)
    e0 = vhat / 2

    def conc(phi, zs):
        g = dc[1:M] * (e0 + np.diff(phi) / dc[1:M])
        ratio = (1 - zs * g / 2) / (1 + zs * g / 2)
        c = np.concatenate([[1.0], np.cumprod(ratio)])
        return c * 2.0 / np.sum(c * dn)

    def lap(phi):
        ext = np.concatenate([[0.0], phi, [0.0]])
        flux = np.diff(ext) / dc
        return np.diff(flux) / dn

    def res(phi):
        return lap(phi) + (conc(phi, 1) - conc(phi, -1)) / (2 * lam ** 2)

    phi0 = np.zeros(M)
    phi = fsolve(res, phi0, xtol=1e-13, maxfev=20000)
    assert np.max(np.abs(res(phi))) < 1e-8
    return phi, conc(phi, 1), conc(phi, -1)


def _continuous_pb(vhat, lam):
    """Phi'' = (A/lam^2) sinh(Phi), Phi(0) = 0, Phi(1) = vhat/2, with c+- =
    A exp(-+Phi) and total mass 2 on [-1, 1] (odd symmetry, solved on [0, 1])."""
    def f(y, s, p):
        return np.vstack([s[1], p[0] / lam ** 2 * np.sinh(s[0]), np.cosh(s[0])])

    def bc(sa, sb, p):
        return np.array([sa[0], sb[0] - vhat / 2, sa[2], sb[2] * p[0] - 1.0])

    y = np.concatenate([np.linspace(0, 0.9, 50), 1 - np.geomspace(0.1, 1e-4, 200)])
    y = np.unique(np.append(y, 1.0))
    guess = np.vstack([vhat / 2 * np.sinh(y / lam) / np.sinh(1 / lam),
                       vhat / 2 / lam * np.cosh(y / lam) / np.sinh(1 / lam), y])
    sol = solve_bvp(f, bc, y, guess, p=[1.0], tol=1e-10, max_nodes=200000)
    assert sol.success
    return sol


def test_poisson_boltzmann_double_layer(oracle_mod):
    vhat, lam = 5.0, 0.1
    o = _quiet(oracle_mod, vhat=vhat, debye=lam)
    o.run(36000)  # t = 6 diffusion times of the gap at Re Sc = 1
    phi = o.field("phi")[:, 0, 0].copy()
    cp = o.field("cp")[:, 0, 0].copy()
    cm = o.field("cm")[:, 0, 0].copy()
    jp, jm, _, _ = o.ion_flux()
    assert np.max(np.abs(jp)) < 1e-9 and np.max(np.abs(jm)) < 1e-9
    # (i) equals the discrete stationary state
    ph_d, cp_d, cm_d = _discrete_pb(o.yn, o.yc, o.dn, o.dc, vhat, lam)
    assert np.max(np.abs(phi - ph_d)) < 1e-9 * vhat
    assert np.max(np.abs(cp - cp_d)) < 1e-9 * cp.max()
    assert np.max(np.abs(cm - cm_d)) < 1e-9 * cm.max()
    # (iii) c+(y) = c-(-y), Phi odd
    assert np.max(np.abs(cp - cm[::-1])) < 1e-10 * cp.max()
    assert np.max(np.abs(phi + phi[::-1])) < 1e-10 * vhat
    # exponential double layers: cations gather at the low-potential wall
    assert cp[0] > 5 and cp[-1] < 0.2 and cm[-1] > 5
    # osmotic balance of the Coulomb force: p - K (c+ + c-) uniform for sF = -1
    K = oracle_mod.coulomb_k(re=1.0, sc=1.0, beta=0.5, debye=lam)
    p = o.field("p")[:, 0, 0]
    osm = p - K * (cp + cm)
    assert np.ptp(osm) < 1e-10 * K * np.ptp(cp + cm)
    # the printed sign (sF = +1) flips the balance: p + K (c+ + c-) uniform
    o2 = _quiet(oracle_mod, vhat=vhat, debye=lam, force_sign=1.0)
    o2.set_state(cp=o.field("cp"), cm=o.field("cm"), phi=o.field("phi"))
    o2.run(30)
    osm2 = o2.field("p")[:, 0, 0] + K * (cp + cm)
    assert np.ptp(osm2) < 1e-9 * K * np.ptp(cp + cm)


def test_poisson_boltzmann_converges_to_continuum(oracle_mod):
    """(ii) The discrete stationary double layer converges at second order to
    the continuous Poisson-Boltzmann solution."""
    vhat, lam = 5.0, 0.1
    sol = _continuous_pb(vhat, lam)
    A = sol.p[0]
    errs = []
    for ny in (33, 65, 129):
        o = oracle_mod.Oracle(nx=1, ny=ny, nz=1, stretch=1.5)
        ph, cp, _ = _discrete_pb(o.yn, o.yc, o.dn, o.dc, vhat, lam)
        yc = o.yc
        Phi_c = np.sign(yc) * sol.sol(np.abs(yc))[0]
        errs.append(np.max(np.abs(vhat / 2 * yc + ph - Phi_c)))
        assert np.max(np.abs(cp - A * np.exp(-Phi_c))) < 0.05 * cp.max()
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), errs


def test_debye_hueckel_limit(oracle_mod):
    """Small voltage: Phi = (vhat/2) sinh(y/lam)/sinh(1/lam), c+- = exp(-+Phi)."""
    vhat, lam = 0.01, 0.1
    o = _quiet(oracle_mod, ny=65, vhat=vhat, debye=lam, dt=2e-3)
    o.run(9000)  # t = 6
    yc = o.yc
    Phi = vhat / 2 * yc + o.field("phi")[:, 0, 0]
    dh = vhat / 2 * np.sinh(yc / lam) / np.sinh(1 / lam)
    assert np.max(np.abs(Phi - dh)) < 3e-3 * vhat / 2
    cp = o.field("cp")[:, 0, 0]
    assert np.max(np.abs(cp - np.exp(-dh))) < 3e-3 * vhat / 2
    cm = o.field("cm")[:, 0, 0]
    assert np.max(np.abs(cm - np.exp(dh))) < 3e-3 * vhat / 2


# --------------------------------------------------------------------------
# time accuracy
# --------------------------------------------------------------------------

def _rk3_x_mode(oracle_mod, dt, T=1.0, eps=0.1):
    o = oracle_mod.Oracle(nx=8, ny=5, nz=2, re=1.0, sc=1.0, vhat=0.0, u_top=0.0, u_bot=0.0, dt=dt)
    o.init(0, 0.0, 0.0)
    xc = (np.arange(8) + 0.5) * o.dx
    c = 1 + eps * np.cos(2 * np.pi * xc / o.cfg.lx)
    o.set_state(cp=np.broadcast_to(c, o.shape), cm=np.broadcast_to(c, o.shape))
    o.solve_potential()
    o.run(int(round(3 * T / dt)))
    k2 = (2 - 2 * np.cos(2 * np.pi / 8)) / o.dx ** 2
    exact = 1 + eps * np.exp(-k2 * T) * np.cos(2 * np.pi * xc / o.cfg.lx)
    return np.max(np.abs(o.field("cp")[2, 1] - exact))


def test_runge_kutta_third_order(oracle_mod):
    errs = [_rk3_x_mode(oracle_mod, dt) for dt in (0.2, 0.1, 0.05)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 2.8) and np.all(orders < 3.3), (errs, orders)


def _eigvec(o, kind):
    n = o.M
    L = np.zeros((n, n))
    for q in range(n):
        e = np.zeros(o.shape)
        e[q] = 1.0
        L[:, q] = o.apply_ly(e, kind, 0.0, 0.0)[:, 0, 0]
    w, V = np.linalg.eig(L)
    order = np.argsort(-w.real)
    idx = order[1] if kind == 0 else order[0]  # skip the constant Neumann mode
    return -w[idx].real, V[:, idx].real / np.max(np.abs(V[:, idx].real))


def _cn_decay(oracle_mod, dt, field, T=0.5, eps=0.1):
    o = oracle_mod.Oracle(nx=1, ny=17, nz=1, re=1.0, sc=1.0, vhat=0.0, u_top=0.0, u_bot=0.0, dt=dt)
    o.init(0, 0.0, 0.0)
    kind = 0 if field == "cp" else 1
    mu, e = _eigvec(o, kind)
    prof = e[:, None, None] * np.ones(o.shape)
    if field == "cp":
        o.set_state(cp=1 + eps * prof, cm=1 + eps * prof)
        o.solve_potential()
        base = 1.0
    else:
        o.set_state(w=eps * prof)
        base = 0.0
    o.run(int(round(3 * T / dt)))
    exact = base + eps * np.exp(-mu * T) * e
    return np.max(np.abs(o.field(field)[:, 0, 0] - exact))


@pytest.mark.parametrize("field", ["cp", "w"])
def test_crank_nicolson_second_order(oracle_mod, field):
    errs = [_cn_decay(oracle_mod, dt, field) for dt in (0.02, 0.01, 0.005)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.85) and np.all(orders < 2.3), (errs, orders)


def _budget_residual(oracle_mod, dt, T=0.06):
    oracle_mod.set_threads(8)
    o = oracle_mod.Oracle(nx=16, ny=17, nz=8, re=100.0, debye=0.1, vhat=5.0, dt=dt)
    o.init(3, 0.05, 1e-2)
    alphas = [8 / 15, 2 / 15, 1 / 3]
    ke0 = o.kinetic_energy()
    ww, dis, fw = o.energy_terms()
    rate = ww - dis + fw
    integral = 0.0
    for s in range(int(round(3 * T / dt))):
        a = alphas[s % 3]
        o.substep()
        ww, dis, fw = o.energy_terms()
        new = ww - dis + fw
        integral += 0.5 * (rate + new) * a * dt
        rate = new
    return abs(o.kinetic_energy() - ke0 - integral), abs(integral)


def test_kinetic_energy_budget_closes(oracle_mod):
    res = [_budget_residual(oracle_mod, dt) for dt in (4e-3, 2e-3, 1e-3)]
    r = np.array([x[0] for x in res])
    assert r[-1] < 1e-3 * res[-1][1]
    orders = np.log2(r[:-1] / r[1:])
    assert np.all(orders > 1.7), (r, orders)


# --------------------------------------------------------------------------
# pi-rotation symmetry of plane Couette flow about the z axis
# --------------------------------------------------------------------------

def _rotate(st):
    """(x, y, z) -> (-x, -y, z): u, v, phi change sign, w keeps it, c+ <-> c-."""
    def cen(a):
        return a[::-1, :, ::-1]

    def xface(a):
        return np.roll(a[::-1, :, ::-1], 1, axis=2)

    v = np.zeros_like(st["v"])
    v[1:] = -st["v"][1:][::-1, :, ::-1]
    return dict(u=-xface(st["u"]), v=v, w=cen(st["w"]), cp=cen(st["cm"]), cm=cen(st["cp"]),
                phi=-cen(st["phi"]), p=cen(st["p"]))


def test_pi_rotation_symmetry_preserved(oracle_mod):
    oracle_mod.set_threads(8)
    o = oracle_mod.Oracle(nx=16, ny=17, nz=12, re=200.0, vhat=6.0, debye=0.15, dt=2e-3)
    o.init(11, 0.05, 1e-2)
    st = o.state()
    rot = _rotate(st)
    sym = {k: 0.5 * (st[k] + rot[k]) for k in ("u", "v", "w", "cp", "cm")}
    o.set_state(**sym, p=np.zeros(o.shape))
    o.solve_potential()
    st0 = o.state()
    r0 = _rotate(st0)
    for k in ("u", "v", "w", "cp", "cm", "phi"):
        assert np.max(np.abs(st0[k] - r0[k])) < 1e-13 * max(1.0, np.max(np.abs(st0[k])))
    o.run(30)
    st1 = o.state()
    r1 = _rotate(st1)
    for k in st1:
        scale = max(1e-3, np.max(np.abs(st1[k])))
        assert np.max(np.abs(st1[k] - r1[k])) < 1e-11 * scale, k
    # and a non-symmetric start does not stay symmetric (the test has teeth)
    o.init(11, 0.05, 1e-2)
    o.run(3)
    st2 = o.state()
    assert np.max(np.abs(st2["u"] - _rotate(st2)["u"])) > 1e-4


# --------------------------------------------------------------------------
# the fractional step equals the unsplit Crank-Nicolson momentum equation
# --------------------------------------------------------------------------

def test_fractional_step_matches_unsplit_momentum_equation(oracle_mod):
    """With the pressure update p += psi - (alpha dt / 2 Re) L_y psi, one
    substep satisfies, exactly in the rows where G_x and L_y commute,
      u1 - u0 = dt (gamma H^k + zeta H^{k-1}) - alpha dt G_x p1
                + (alpha dt / 2 Re) L_y (u1 + u0)."""
    oracle_mod.set_threads(8)
    re, dt = 50.0, 4e-3
    o = oracle_mod.Oracle(nx=12, ny=17, nz=8, re=re, vhat=4.0, debye=0.15, dt=dt)
    o.init(2, 0.1, 1e-2)
    gam = [8 / 15, 5 / 12, 3 / 4]
    zet = [0.0, -17 / 60, -5 / 12]
    for _ in range(4):  # check stages 2, 3, 1, 2
        o.substep()
        k = o.stage
        a = gam[k] + zet[k]
        u0 = o.field("u").copy()
        w0 = o.field("w").copy()
        hold_u, hold_w = o.hold(0).copy(), o.hold(2).copy()
        h = o.explicit_terms()
        o.substep()
        u1, w1, p1 = o.field("u").copy(), o.field("w").copy(), o.field("p").copy()
        gx, _, gz = o.gradient(p1)
        for q0, q1, hk, hkm, g, lo, hi in ((u0, u1, h["u"], hold_u, gx, -1.0, 1.0),
                                           (w0, w1, h["w"], hold_w, gz, 0.0, 0.0)):
            ly = o.apply_ly(q1 + q0, 1, 2 * lo, 2 * hi)
            rhs = dt * (gam[k] * hk + zet[k] * hkm) - a * dt * g + a * dt / (2 * re) * ly
            res = (q1 - q0 - rhs)[1:-1]
            assert np.max(np.abs(res)) < 1e-14, (k, np.max(np.abs(res)))
