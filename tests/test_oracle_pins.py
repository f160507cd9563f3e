"""Pins of the FP64 oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: closed
forms, exact solutions of the continuous equations, conservation
invariants, exact polynomial reproduction, or convergence at the design
order.  A plausible slip anywhere in the oracle (dropped term, wrong sign,
wrong index, transposed operand) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import problems as P
from tests import exact

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def setup_module(module):
    oracle.build(force=False)


# --------------------------------------------------------------- RK3 (Sec. 2.2)
def test_rk3_linear_stability_polynomial():
    """One Wray RK3 step on dw/dt = lam w is exactly 1 + z + z^2/2 + z^3/6.

    Any three-stage third-order scheme has this amplification factor; the
    printed +17/60 would give a different cubic."""
    for lam, dt in [(-1.0, 0.1), (-3.7, 0.21), (2.0, 0.05), (-0.5, 1.3)]:
        w = np.array([1.0])
        rprev = np.zeros(1)
        for l in range(3):
            r = lam * w
            w = oracle.rk_stage(w, r, rprev, dt, l)
            rprev = r
        z = lam * dt
        assert abs(w[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14 * max(1.0, abs(w[0]))


def test_rk3_third_order_nonlinear():
    """dw/dt = -w^2, w(0)=1 -> 1/(1+t): global error falls ~8x per halving of dt."""
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        w = np.array([1.0])
        for _ in range(n):
            rprev = np.zeros(1)
            for l in range(3):
                r = -w * w
                w = oracle.rk_stage(w, r, rprev, dt, l)
                rprev = r
        errs.append(abs(w[0] - 0.5))
    assert 7.0 < errs[0] / errs[1] < 9.0
    assert 7.0 < errs[1] / errs[2] < 9.0


# --------------------------------------------------------------- WENO5 (Sec. 2.1)
def _cell_avgs(poly, xs, h):
    """Exact cell averages of a numpy poly1d over [x-h/2, x+h/2]."""
    P_ = np.polyint(poly)
    return (P_(xs + h / 2) - P_(xs - h / 2)) / h


def test_weno5_reproduces_quadratics_exactly():
    rng = np.random.default_rng(0)
    for _ in range(20):
        c = rng.normal(size=3)
        poly = np.poly1d(c)
        h = rng.uniform(0.05, 0.5)
        x0 = rng.uniform(-1, 1)
        xs = x0 + h * np.arange(-2, 3)
        v = _cell_avgs(poly, xs, h)
        val = oracle.weno5(v)
        assert abs(val - poly(x0 + h / 2)) < 1e-13 * max(1.0, abs(poly(x0 + h / 2)))


def _weno5_from_polynomials(v, h=1.0, eps=1e-6):
    """WENO5-JS rebuilt from its definition: the three quadratic candidates
    matching the cell averages of their stencils, smoothness indicators
    beta_k = sum_l h^(2l-1) int_cell (p_k^(l))^2 dx, weights d/(eps+beta)^2."""
    P_ = np.polynomial.Polynomial
    centers = h * np.arange(-2, 3)
    x_face = h / 2
    stencils = [(0, 1, 2), (1, 2, 3), (2, 3, 4)]
    dlin = [0.1, 0.6, 0.3]
    qs, betas = [], []
    for st in stencils:
        A = np.zeros((3, 3))
        for r, c in enumerate(st):
            for pw in range(3):
                a, b = centers[c] - h / 2, centers[c] + h / 2
                A[r, pw] = (b ** (pw + 1) - a ** (pw + 1)) / ((pw + 1) * h)
        coef = np.linalg.solve(A, np.array([v[c] for c in st]))
        p = P_(coef)
        qs.append(p(x_face))
        beta = 0.0
        for l in (1, 2):
            dp = p.deriv(l)
            integ = (dp * dp).integ()
            beta += h ** (2 * l - 1) * (integ(h / 2) - integ(-h / 2))
        betas.append(beta)
    al = np.array(dlin) / (eps + np.array(betas)) ** 2
    return float(al @ np.array(qs) / al.sum())


def test_weno5_matches_definition_from_candidate_polynomials():
    rng = np.random.default_rng(7)
    for scale in (1e-3, 1.0, 30.0):
        for _ in range(200):
            v = scale * rng.normal(size=5)
            ref = _weno5_from_polynomials(v)
            assert abs(oracle.weno5(v) - ref) <= 1e-12 * max(1.0, np.abs(v).max())


def test_weno5_fifth_order_on_smooth_data():
    """Face value from cell averages of exp(sin x): error ratio ~32 per halving."""
    f = lambda x: np.exp(np.sin(x))
    errs = []
    for h in (0.2, 0.1, 0.05):
        x0 = 0.3
        xs = x0 + h * np.arange(-2, 3)
        # cell averages by high-order Gauss quadrature
        gx, gw = np.polynomial.legendre.leggauss(12)
        v = np.array([np.sum(gw * f(xc + 0.5 * h * gx)) / 2 for xc in xs])
        errs.append(abs(oracle.weno5(v) - f(x0 + h / 2)))
    assert errs[0] / errs[1] > 20 and errs[1] / errs[2] > 25


def test_weno5_non_oscillatory_at_a_jump():
    v = np.array([1.0, 1.0, 1.0, 0.0, 0.0])
    val = oracle.weno5(v)
    assert -1e-6 < val < 1.0 + 1e-6
    assert abs(val - 1.0) < 1e-3  # upwind smooth stencil dominates
    v = np.array([1.0, 1.0, 0.0, 0.0, 0.0])
    assert abs(oracle.weno5(v)) < 1e-3


# --------------------------------------------------------------- eigenvectors
def _euler_flux(wv, d, g):
    rho = wv[0]
    vel = wv[1:4] / rho
    p = (g - 1) * (wv[4] - 0.5 * rho * np.dot(vel, vel))
    f = np.zeros(5)
    f[0] = rho * vel[d]
    f[1:4] = rho * vel[d] * vel
    f[1 + d] += p
    f[4] = vel[d] * (wv[4] + p)
    return f


@pytest.mark.parametrize("d", [0, 1, 2])
def test_eigenvectors_diagonalise_flux_jacobian(d):
    g = 1.4
    rng = np.random.default_rng(d)
    for _ in range(5):
        rho = rng.uniform(0.5, 2)
        vel = rng.uniform(-1, 1, 3)
        p = rng.uniform(0.5, 2)
        wv = np.array([rho, *(rho * vel), p / (g - 1) + 0.5 * rho * vel @ vel])
        Ht = (wv[4] + p) / rho
        R, L = oracle.eigenvectors(g, d, *vel, Ht)
        assert np.abs(L @ R - np.eye(5)).max() < 1e-13
        c = math.sqrt(g * p / rho)
        lam = np.array([vel[d] - c, vel[d], vel[d], vel[d], vel[d] + c])
        # flux Jacobian by central differences of the continuous flux
        J = np.zeros((5, 5))
        for k in range(5):
            e = np.zeros(5)
            e[k] = 1e-6 * max(1.0, abs(wv[k]))
            J[:, k] = (_euler_flux(wv + e, d, g) - _euler_flux(wv - e, d, g)) / (2 * e[k])
        assert np.abs(R @ np.diag(lam) @ L - J).max() < 1e-7


# --------------------------------------------------------------- manufactured RHS
def _manufactured_problem(n, stretched=False, viscous=True):
    L = 2 * math.pi
    if stretched:
        y, ye, yee = P.periodic_stretched_y(n, L, amp=0.3)
    else:
        y, ye, yee = P.uniform_periodic_y(n, L)
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(x, y, x, indexing="ij")
    g, Rg, Pr, mu, S = 1.4, 1.0 / (1.4 * 0.5 ** 2), 0.72, 0.05, 0.368
    prim, euler, visc = exact.manufactured_rhs(g, Rg, Pr, mu, S)
    rho, u, v, w, p = exact.eval_fields(prim, X, Y, Z)
    w0 = P.conserved_from_primitive(rho, u, v, w, p, g)
    pr = P.Problem(name="mms", nx=n, ny=n, nz=n, lx=L, lz=L, y=y, y_eta=ye, y_etaeta=yee,
                   gamma=g, Pr=Pr, R_gas=Rg, mu_ref=mu, T_ref=1.0, S_suth=S, viscous=viscous,
                   sensor_mode=P.SENSOR_OFF, forcing=False, w0=w0)
    return pr, exact.eval_fields(euler, X, Y, Z), exact.eval_fields(visc, X, Y, Z)


@pytest.mark.parametrize("stretched", [False, True])
def test_inviscid_operator_fourth_order_against_exact(stretched):
    errs = []
    for n in (16, 32, 64):
        pr, ex_e, _ = _manufactured_problem(n, stretched)
        r = oracle.rhs(pr, terms=oracle.T_CONV | oracle.T_PRES)
        errs.append([np.abs(r[m] - ex_e[m]).max() / np.abs(ex_e[m]).max() for m in range(5)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert (ratios[-1] > 13.0).all(), (errs, ratios)
    assert errs[-1].max() < 2e-4


@pytest.mark.parametrize("stretched", [False, True])
def test_viscous_operator_fourth_order_against_divergence_form(stretched):
    """Laplacian-form viscous and heat terms against the exact divergence form."""
    errs = []
    for n in (16, 32, 64):
        pr, _, ex_v = _manufactured_problem(n, stretched)
        r = oracle.rhs(pr, terms=oracle.T_VISC)
        errs.append([np.abs(r[m] - ex_v[m]).max() / np.abs(ex_v[m]).max() for m in range(1, 5)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert (ratios[-1] > 13.0).all(), (errs, ratios)
    assert errs[-1].max() < 5e-4


def test_pressure_flux_difference_is_central_derivative():
    """With only the pressure part, R_mom = -D1 p exactly (4th-order central)."""
    n = 12
    pr, _, _ = _manufactured_problem(n)
    r = oracle.rhs(pr, terms=oracle.T_PRES)
    w0 = pr.w0
    rho = w0[0]
    ke = 0.5 * (w0[1] ** 2 + w0[2] ** 2 + w0[3] ** 2) / rho
    p = (pr.gamma - 1) * (w0[4] - ke)
    h = pr.lx / n
    def d1(f, ax, h):
        return (2 / 3 * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
                - 1 / 12 * (np.roll(f, -2, ax) - np.roll(f, 2, ax))) / h
    assert np.abs(r[1] + d1(p, 2, h)).max() < 1e-12 * np.abs(p).max() / h
    assert np.abs(r[2] + d1(p, 1, h)).max() < 1e-12 * np.abs(p).max() / h
    assert np.abs(r[3] + d1(p, 0, h)).max() < 1e-12 * np.abs(p).max() / h
    assert np.abs(r[0]).max() == 0 and np.abs(r[4]).max() == 0


# --------------------------------------------------------------- invariants
def test_uniform_state_has_zero_rhs():
    pr = P.taylor_green(8)
    w0 = np.zeros_like(pr.w0)
    w0[:] = P.conserved_from_primitive(1.3, 0.2, -0.1, 0.3, 2.0, 1.4)[:, None, None, None]
    for mode in (0, 2):
        r = oracle.rhs(P.with_state(pr, w0, sensor_mode=mode))
        assert np.abs(r).max() < 1e-13


@pytest.mark.parametrize("mode", [P.SENSOR_OFF, P.SENSOR_HYBRID, P.SENSOR_WENO_ALL])
def test_periodic_inviscid_conservation(mode):
    """Flux form: sum of R dV vanishes to round-off for all five equations."""
    pr = P.decaying_turbulence(16, mach=1.5, re=500.0, seed=5)
    pr = P.with_state(pr, pr.w0, viscous=False, sensor_mode=mode, theta_star=0.05)
    r = oracle.rhs(pr)
    for m in range(5):
        scale = np.abs(r[m]).max() * r[m].size
        assert abs(r[m].sum()) < 1e-13 * scale, (m, r[m].sum(), scale)


def test_periodic_inviscid_conservation_stretched():
    pr, _, _ = _manufactured_problem(16, stretched=True, viscous=False)
    for mode in (0, 2):
        r = oracle.rhs(P.with_state(pr, pr.w0, sensor_mode=mode))
        for m in range(5):
            tot = (r[m] * pr.y_eta[None, :, None]).sum()
            scale = (np.abs(r[m]) * pr.y_eta[None, :, None]).sum()
            assert abs(tot) < 1e-13 * scale


def test_kinetic_energy_preservation_of_convective_terms():
    """Split-form central convective terms add nothing to the discrete kinetic
    energy: sum(u . C_mom - |u|^2/2 C_mass) dV = 0 to round-off."""
    pr = P.decaying_turbulence(16, mach=0.5, re=500.0, seed=3)
    # add density/temperature variation so the identity is non-trivial
    rng = np.random.default_rng(1)
    w0 = pr.w0.copy()
    fac = 1.0 + 0.3 * rng.uniform(-1, 1, w0.shape[1:])
    w0 *= fac[None]
    pr = P.with_state(pr, w0, viscous=False, sensor_mode=P.SENSOR_OFF)
    c = oracle.rhs(pr, terms=oracle.T_CONV)
    rho = w0[0]
    u = w0[1:4] / rho
    dk = (u * c[1:4]).sum(axis=0) - 0.5 * (u * u).sum(axis=0) * c[0]
    scale = np.abs((u * c[1:4]).sum(axis=0)).sum()
    assert abs(dk.sum()) < 1e-13 * scale
    # a divergence-form (non-split) flux would not satisfy it: sanity of the test
    assert scale > 1.0


def test_channel_walls_conserve_mass_and_balance_wall_pressure():
    """Staggered walls carry no convective flux: sum R_rho dV = 0; the wall-normal
    momentum balance reduces to the two wall pressure fluxes (7 p0 - p1)/6."""
    pr = P.small_channel(16, 16, 8)
    pr = P.with_state(pr, pr.w0, viscous=False, forcing=False, sensor_mode=P.SENSOR_OFF)
    r = oracle.rhs(pr)
    ye = pr.y_eta[None, :, None]
    assert abs((r[0] * ye).sum()) < 1e-13 * (np.abs(r[0]) * ye).sum()
    w0 = pr.w0
    rho = w0[0]
    p = (pr.gamma - 1) * (w0[4] - 0.5 * (w0[1] ** 2 + w0[2] ** 2 + w0[3] ** 2) / rho)
    pw_lo = (7 * p[:, 0, :] - p[:, 1, :]) / 6
    pw_hi = (7 * p[:, -1, :] - p[:, -2, :]) / 6
    deta = 1.0 / pr.ny
    lhs = (r[2] * ye * deta).sum()
    rhs = (pw_lo - pw_hi).sum()
    assert abs(lhs - rhs) < 1e-12 * np.abs(pw_lo).sum()


def test_wall_at_rest_isothermal_is_steady():
    pr = P.small_channel(12, 16, 8)
    shape = pr.w0.shape[1:]
    w0 = P.conserved_from_primitive(np.ones(shape), np.zeros(shape), np.zeros(shape),
                                    np.zeros(shape), np.full(shape, pr.R_gas), pr.gamma)
    r = oracle.rhs(P.with_state(pr, w0, forcing=False))
    assert np.abs(r).max() < 1e-12


def test_forcing_keeps_mass_flow_constant():
    pr = P.small_channel(16, 16, 8, nsteps=5)
    ye = pr.y_eta[None, :, None]
    r, _, _, _, f = oracle.rhs(pr, want_flags=True)
    assert abs((r[1] * ye).sum()) < 1e-13 * (np.abs(r[1]) * ye).sum()
    # energy receives exactly f * u at each node
    r_nf = oracle.rhs(pr, terms=oracle.T_ALL & ~oracle.T_FORCE)
    u = pr.w0[1] / pr.w0[0]
    assert np.abs(r[4] - r_nf[4] - f * u).max() < 1e-12 * np.abs(r[4]).max()
    assert np.abs(r[1] - r_nf[1] - f).max() < 1e-12 * np.abs(r[1]).max()
    m0 = (pr.w0[1] * ye).sum()
    w = oracle.advance(pr, 5)
    assert abs((w[1] * ye).sum() - m0) < 1e-13 * abs(m0)


# --------------------------------------------------------------- sensor
def test_sensor_closed_form_for_compression_wave():
    """u = A sin x: D1 gives div = kappa A cos x exactly, curl = 0, so
    theta = max(-kappa A cos x / sqrt((kappa A cos x)^2 + eps), 0)."""
    n = 16
    pr = P.taylor_green(n)
    L = 2 * math.pi
    h = L / n
    x = np.arange(n) * h
    A, eps = 0.7, 0.3
    shape = pr.w0.shape[1:]
    u = np.broadcast_to(A * np.sin(x)[None, None, :], shape)
    w0 = P.conserved_from_primitive(np.ones(shape), u, np.zeros(shape), np.zeros(shape),
                                    np.full(shape, 5.0), 1.4)
    pr2 = P.with_state(pr, w0, sensor_mode=P.SENSOR_HYBRID, sensor_eps=eps, theta_star=0.5)
    _, theta, nfl, ifl, _ = oracle.rhs(pr2, want_flags=True)
    kappa = (4 / 3 * math.sin(h) - 1 / 6 * math.sin(2 * h)) / h
    dv = kappa * A * np.cos(x)
    th = np.maximum(-dv / np.sqrt(dv * dv + eps), 0.0)
    assert np.abs(theta - th[None, None, :]).max() < 1e-14
    assert (nfl == (theta > 0.5)).all()
    # interface flags in x: OR over nodes i-1..i+2 (periodic)
    f = (th > 0.5).astype(np.uint8)
    ix = f | np.roll(f, 1) | np.roll(f, -1) | np.roll(f, -2)
    assert ((ifl & 1) == ix[None, None, :]).all()
    # no compression along y or z: those interfaces stay central except where
    # the node itself (OR neighbours along y/z, same x) is flagged
    assert (((ifl >> 1) & 1) == f[None, None, :]).all()


def test_sensor_vanishes_for_solenoidal_fields():
    n = 16
    pr = P.taylor_green(n)
    pr2 = P.with_state(pr, pr.w0, sensor_mode=P.SENSOR_HYBRID, theta_star=0.0)
    # the Taylor-Green velocity is divergence free; D1 keeps it so to round-off
    _, theta, _, _, _ = oracle.rhs(pr2, want_flags=True)
    assert theta.max() < 1e-12


# --------------------------------------------------------------- Sod (exact Riemann)
def _sod_run(n, axis):
    pr = P.sod_tube(n, axis=axis)
    h = 2.0 / n
    t_end = 0.2
    dt = 0.2 * h  # CFL ~ 0.4 at max speed ~1.75+ (sound speed 1.18 + |u| 0.93)
    nsteps = int(round(t_end / dt))
    w = oracle.advance(pr, nsteps, dt_fixed=dt)
    line = [0, 0, 0]
    line[2 - axis] = slice(None)
    rho = w[0][tuple(line)]
    s = (np.arange(n) + 0.5) * h
    ex = exact.riemann_sample(P.SOD_LEFT, P.SOD_RIGHT, (s - 1.0) / t_end)
    mir = exact.riemann_sample(P.SOD_RIGHT, P.SOD_LEFT, np.where(s < 1.0, s, s - 2.0) / t_end)
    exact_rho = np.where(np.abs(s - 1.0) < 0.6, ex[0], mir[0])
    return s, rho, exact_rho, w


def test_exact_riemann_solver_matches_tabulated_sod_solution():
    """The exact solver used as reference below reproduces the star state of
    Sod's problem tabulated in Toro's textbook (tests/golden/sod_star_state.txt)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sod_star_state.txt")
    ref = {k: float(v) for k, v in (line.split() for line in open(path)
                                     if line.strip() and not line.startswith("#"))}
    ps, us = exact.riemann_star(P.SOD_LEFT, P.SOD_RIGHT)
    assert abs(ps - ref["p_star"]) < 6e-6 and abs(us - ref["u_star"]) < 6e-6
    eps = 1e-6
    rho_l = exact.riemann_sample(P.SOD_LEFT, P.SOD_RIGHT, np.array([us - eps]))[0][0]
    rho_r = exact.riemann_sample(P.SOD_LEFT, P.SOD_RIGHT, np.array([us + eps]))[0][0]
    assert abs(rho_l - ref["rho_star_left"]) < 6e-6 and abs(rho_r - ref["rho_star_right"]) < 6e-6


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sod_shock_tube_against_exact_riemann(axis):
    errs = []
    for n in (100, 200):
        s, rho, ex, w = _sod_run(n, axis)
        errs.append(np.mean(np.abs(rho - ex)) * 2.0)
        # shock position: exact shock at x = 1 + 1.7522 * 0.2; density between
        # post-shock (0.2656) and pre-shock (0.125) crosses the mid value within 2 cells
    assert errs[1] < errs[0] and errs[1] < 0.02, errs
    ps, us = exact.riemann_star(P.SOD_LEFT, P.SOD_RIGHT)
    rs = 0.125 * (ps / 0.1 + 1 / 6) / (ps / 0.1 / 6 + 1)
    shock_speed = us * rs / (rs - 0.125)  # mass conservation across the shock
    xs = 1.0 + shock_speed * 0.2
    mid = 0.5 * (rs + 0.125)
    idx = np.where((s > 1.3) & (s < 1.5) & (rho < mid))[0][0]
    assert abs(s[idx] - xs) < 2 * (2.0 / 200)
    # transverse momentum stays exactly zero
    assert np.abs(w[1 + (axis + 1) % 3]).max() < 1e-14


def test_hybrid_sensor_fires_at_shock_not_in_rarefaction():
    n = 200
    pr = P.sod_tube(n, axis=0, sensor_mode=P.SENSOR_HYBRID, theta_star=0.3)
    h = 2.0 / n
    w = oracle.advance(pr, 40, dt_fixed=0.2 * h)  # t = 0.08
    _, theta, nfl, _, _ = oracle.rhs(P.with_state(pr, w), want_flags=True)
    s = (np.arange(n) + 0.5) * h
    t = 40 * 0.2 * h
    ps, us = exact.riemann_star(P.SOD_LEFT, P.SOD_RIGHT)
    rs = 0.125 * (ps / 0.1 + 1 / 6) / (ps / 0.1 / 6 + 1)
    xs = 1.0 + us * rs / (rs - 0.125) * t
    th = theta[0, 0]
    near_shock = np.abs(s - xs) < 3 * h
    assert th[near_shock].max() > 0.9
    # rarefaction fan: expansion, div u > 0 -> theta = 0
    c = math.sqrt(1.4)
    fan = (s > 1.0 - c * t + 2 * h) & (s < 1.0 - 0.3 * t)
    assert th[fan].max() == 0.0


# --------------------------------------------------------------- isentropic vortex
@pytest.mark.parametrize("plane", ["xy", "yz"])
def test_isentropic_vortex_design_order(plane):
    errs = []
    t_end, dt = 0.5, 0.01
    for n in (32, 64):
        pr = P.isentropic_vortex(n, plane=plane)
        w = oracle.advance(pr, int(round(t_end / dt)), dt_fixed=dt)
        ex = P.isentropic_vortex(n, plane=plane, t=t_end).w0
        errs.append(np.abs(w[0] - ex[0]).max())
    rate = math.log2(errs[0] / errs[1])
    assert rate > 3.4, (errs, rate)


# --------------------------------------------------------------- time step rule
def test_dt_rule_uniform_state():
    pr = P.taylor_green(8)
    shape = pr.w0.shape[1:]
    u, v, w, rho, p = 0.3, -0.2, 0.1, 1.2, 2.0
    w0 = P.conserved_from_primitive(np.full(shape, rho), np.full(shape, u), np.full(shape, v),
                                    np.full(shape, w), np.full(shape, p), 1.4)
    pr2 = P.with_state(pr, w0, viscous=False)
    c = math.sqrt(1.4 * p / rho)
    h = 2 * math.pi / 8
    expect = 0.8 / ((abs(u) + c) / h + (abs(v) + c) / h + (abs(w) + c) / h)
    assert abs(oracle.dt(pr2, cfl=0.8) - expect) < 1e-15 * expect


# --------------------------------------------------------------- shock top input
def test_oblique_shock_relations():
    beta, p21, r21, m2 = P.oblique_shock(2.0, 8.0)
    assert abs(math.degrees(beta) - 37.21) < 0.01
    assert abs(p21 - 1.540) < 1e-3
    assert abs(r21 - 1.358) < 1e-3
    assert abs(m2 - 1.714) < 1e-3


# --------------------------------------------------------------- open boundaries
def _open_box(n=120, nthin=4):
    pr = P.sod_tube(n, axis=0, sensor_mode=P.SENSOR_OFF)
    bcs = list(pr.bcs)
    bcs[P.FACE_XM] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    bcs[P.FACE_XP] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    return P.with_state(pr, pr.w0, bcs=bcs, lx=1.0)


def test_open_boundaries_keep_uniform_flow_steady():
    pr = _open_box()
    shape = pr.w0.shape[1:]
    w0 = P.conserved_from_primitive(np.full(shape, 1.1), np.full(shape, 0.4),
                                    np.full(shape, -0.1), np.zeros(shape),
                                    np.full(shape, 0.9), 1.4)
    bcs = list(pr.bcs)
    prof = np.array([[1.1], [0.4], [-0.1], [0.0], [0.9]]) * np.ones((5, pr.ny))
    bcs[P.FACE_XM] = (P.BC_DIRICHLET, prof)
    for mode in (0, 2):
        r = oracle.rhs(P.with_state(pr, w0, bcs=bcs, sensor_mode=mode))
        assert np.abs(r).max() < 1e-12


def test_characteristic_outflow_lets_acoustic_pulse_leave():
    """Behaviour check (the paper gives no formula for its non-reflecting
    treatment): a right-running acoustic pulse leaves through x+ with less
    than 5% of its amplitude reflected."""
    n = 200
    pr = _open_box(n)
    x = (np.arange(n) + 0.5) / n
    eps = 1e-3
    dp = eps * np.exp(-((x - 0.5) / 0.05) ** 2)
    shape = pr.w0.shape[1:]
    c = 1.0
    p0 = 1.0 / 1.4
    p = p0 + dp
    rho = 1.0 + dp / c ** 2
    u = dp / c
    bc = lambda a: np.broadcast_to(a[None, None, :], shape)
    w0 = P.conserved_from_primitive(bc(rho), bc(u), np.zeros(shape), np.zeros(shape), bc(p), 1.4)
    pr2 = P.with_state(pr, w0)
    h = 1.0 / n
    dt = 0.4 * h
    w = oracle.advance(pr2, int(0.9 / dt), dt_fixed=dt)  # pulse centre reaches x = 1.4
    pp = (pr.gamma - 1) * (w[4] - 0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / w[0])
    assert np.abs(pp - p0).max() < 0.05 * eps


def test_invalid_configurations_are_rejected():
    pr = P.taylor_green(8)
    bcs = list(pr.bcs)
    bcs[P.FACE_XM] = (P.BC_WALL_ADIABATIC, np.zeros(0))  # unpaired periodic + wall on x
    with pytest.raises(oracle.OracleError):
        oracle.rhs(P.with_state(pr, pr.w0, bcs=bcs))
    # a state with negative density is reported, not silently used
    w0 = pr.w0.copy()
    w0[0, 1, 2, 3] = -1.0
    with pytest.raises(oracle.OracleError):
        oracle.rhs(P.with_state(pr, w0))


def test_results_do_not_depend_on_the_thread_count():
    # the oracle's parallel loops write disjoint outputs and reduce only with
    # a bitwise or, so a state after several steps is the same bit for bit
    # on one thread and on all of them
    pr = P.decaying_turbulence(12, mach=0.5, re=500.0, seed=3)
    prev = oracle.set_threads(1)
    try:
        assert oracle.num_threads() == 1
        w1 = oracle.advance(pr, 3, cfl=pr.cfl)
    finally:
        oracle.set_threads(prev)
    assert oracle.num_threads() == prev
    wn = oracle.advance(pr, 3, cfl=pr.cfl)
    assert np.array_equal(w1, wn)
