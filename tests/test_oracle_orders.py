"""Pins of the oracle's scheme-order variants (Sec. 2.1, eq. encflux and the
Laplacian-form viscous terms: order 2L for any L; the WENO reconstruction of
the Jiang-Shu family, order 2r - 1).

Every expected value here is derived independently of the oracle's
coefficient tables: central-difference weights from Taylor (Vandermonde)
systems, WENO candidates and smoothness indicators from polynomials fitted
to cell averages and integrated exactly, design orders from convergence on
smooth fields, conservation and kinetic-energy identities from the flux
form, and the Sod problem from the exact Riemann solution.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import problems as P
from tests import exact
from tests.test_oracle_pins import _manufactured_problem, _sod_run

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def setup_module(module):
    oracle.build(force=False)


def taylor_weights(L, deriv):
    """Exact central weights w_{-L..L} of the derivative `deriv` of order 2L
    (solve sum_l w_l l^k = k! [k == deriv] for k = 0..2L in rationals)."""
    n = 2 * L + 1
    offs = list(range(-L, L + 1))
    A = [[Fraction(o) ** k for o in offs] for k in range(n)]
    b = [Fraction(math.factorial(deriv)) if k == deriv else Fraction(0) for k in range(n)]
    # Gauss-Jordan elimination in exact arithmetic
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [x - fac * y for x, y in zip(M[r], M[c])]
    return {o: M[i][n] for i, o in enumerate(offs)}


def with_orders(pr, central=4, weno=5, **kw):
    return P.with_state(pr, pr.w0, central_order=central, weno_order=weno, **kw)


# --------------------------------------------------------------- WENO family
def _cell_poly(vals, offs):
    """Coefficients (ascending) of the polynomial of degree len-1 whose
    averages over the unit cells centred at offs are vals."""
    n = len(vals)
    A = np.zeros((n, n))
    for row, o in enumerate(offs):
        for m in range(n):
            A[row, m] = ((o + 0.5) ** (m + 1) - (o - 0.5) ** (m + 1)) / (m + 1)
    return np.linalg.solve(A, vals)


def _smoothness(coef):
    """sum_{m>=1} int_{-1/2}^{1/2} (p^(m))^2 dx for unit spacing."""
    Pn = np.polynomial.polynomial
    b = 0.0
    for m in range(1, len(coef)):
        d = Pn.polyder(coef, m)
        I = Pn.polyint(Pn.polymul(d, d))
        b += Pn.polyval(0.5, I) - Pn.polyval(-0.5, I)
    return b


@pytest.mark.parametrize("r", [2, 3, 4])
def test_weno_candidates_and_indicators_match_polynomial_definition(r):
    rng = np.random.default_rng(10 + r)
    for scale in (1e-2, 1.0, 40.0):
        for _ in range(50):
            v = scale * rng.normal(size=2 * r - 1)
            q, beta = oracle.weno_parts(r, v)
            for k in range(r):
                offs = list(range(-r + 1 + k, k + 1))
                coef = _cell_poly(v[k:k + r], offs)
                qk = np.polynomial.polynomial.polyval(0.5, coef)
                bk = _smoothness(coef)
                assert abs(q[k] - qk) <= 1e-12 * scale * 10, (r, k)
                assert abs(beta[k] - bk) <= 1e-11 * max(bk, scale * scale), (r, k, beta[k], bk)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_weno_linear_weights_give_the_full_stencil_reconstruction(r):
    """For data of tiny variation (beta << eps) the nonlinear weights equal
    the linear ones, and the combination must equal the face value of the
    polynomial of degree 2r-2 fitted to all 2r-1 cell averages (the
    optimal-order upwind-biased reconstruction)."""
    rng = np.random.default_rng(3)
    delta = 1e-7
    for _ in range(30):
        g = rng.normal(size=2 * r - 1)
        val = (oracle.weno(r, 1.0 + delta * g) - 1.0) / delta
        coef = _cell_poly(g, list(range(-r + 1, r)))
        ref = np.polynomial.polynomial.polyval(0.5, coef)
        assert abs(val - ref) < 1e-4 * max(1.0, np.abs(g).max()), (r, val, ref)


@pytest.mark.parametrize("r,hs,min_ratio", [(2, (0.2, 0.1, 0.05), 7.0),
                                            (3, (0.2, 0.1, 0.05), 25.0),
                                            (4, (0.1, 0.05, 0.025), 64.0)])
def test_weno_design_order_on_smooth_data(r, hs, min_ratio):
    """Face value from cell averages of exp(sin x) at a non-critical point:
    the error falls by about 2^(2r-1) per halving."""
    f = lambda x: np.exp(np.sin(x))
    gx, gw = np.polynomial.legendre.leggauss(12)
    errs = []
    for h in hs:
        x0 = 0.3
        xs = x0 + h * np.arange(-(r - 1), r)
        v = np.array([np.sum(gw * f(xc + 0.5 * h * gx)) / 2 for xc in xs])
        errs.append(abs(oracle.weno(r, v) - f(x0 + h / 2)))
    assert errs[0] / errs[1] > min_ratio and errs[1] / errs[2] > min_ratio, errs


@pytest.mark.parametrize("r", [2, 4])
def test_weno_non_oscillatory_at_a_jump(r):
    n = 2 * r - 1
    for cut in range(1, n):
        v = np.where(np.arange(n) < cut, 1.0, 0.0)
        val = oracle.weno(r, v)
        assert -1e-6 < val < 1.0 + 1e-6, (r, cut, val)


# --------------------------------------------------------------- central flux of order 2L
@pytest.mark.parametrize("L", [1, 2, 3])
def test_pressure_flux_difference_is_central_derivative_of_order_2L(L):
    """With only the pressure part, R_mom = -D1 p with the exact order-2L
    first-derivative weights (derived here from the Taylor system)."""
    n = 12
    pr, _, _ = _manufactured_problem(n)
    pr = with_orders(pr, central=2 * L)
    r = oracle.rhs(pr, terms=oracle.T_PRES)
    w0 = pr.w0
    ke = 0.5 * (w0[1] ** 2 + w0[2] ** 2 + w0[3] ** 2) / w0[0]
    p = (pr.gamma - 1) * (w0[4] - ke)
    h = pr.lx / n
    wts = taylor_weights(L, 1)

    def d1(f, ax):
        return sum(float(wt) * np.roll(f, -o, ax) for o, wt in wts.items() if o != 0) / h

    for m, ax in ((1, 2), (2, 1), (3, 0)):
        assert np.abs(r[m] + d1(p, ax)).max() < 1e-12 * np.abs(p).max() / h, (L, m)
    assert np.abs(r[0]).max() == 0 and np.abs(r[4]).max() == 0


@pytest.mark.parametrize("L,min_ratio", [(1, 3.5), (3, 50.0)])
def test_inviscid_operator_order_2L_against_exact(L, min_ratio):
    errs = []
    for n in (16, 32, 64):
        pr, ex_e, _ = _manufactured_problem(n, stretched=False, viscous=False)
        r = oracle.rhs(with_orders(pr, central=2 * L), terms=oracle.T_CONV | oracle.T_PRES)
        errs.append([np.abs(r[m] - ex_e[m]).max() / np.abs(ex_e[m]).max() for m in range(5)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert (ratios[-1] > min_ratio).all(), (errs, ratios)


@pytest.mark.parametrize("L,min_ratio", [(1, 3.5), (3, 50.0)])
@pytest.mark.parametrize("stretched", [False, True])
def test_viscous_operator_order_2L_against_divergence_form(L, min_ratio, stretched):
    errs = []
    for n in (16, 32, 64):
        pr, _, ex_v = _manufactured_problem(n, stretched)
        r = oracle.rhs(with_orders(pr, central=2 * L), terms=oracle.T_VISC)
        errs.append([np.abs(r[m] - ex_v[m]).max() / np.abs(ex_v[m]).max() for m in range(1, 5)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert (ratios[-1] > min_ratio).all(), (errs, ratios)


@pytest.mark.parametrize("L", [1, 3])
def test_kinetic_energy_preservation_for_every_L(L):
    """The split form preserves kinetic energy for any L (the identity holds
    pair by pair): sum(u . C_mom - |u|^2/2 C_mass) dV = 0 to round-off."""
    pr = P.decaying_turbulence(16, mach=0.5, re=500.0, seed=3)
    rng = np.random.default_rng(1)
    w0 = pr.w0 * (1.0 + 0.3 * rng.uniform(-1, 1, pr.w0.shape[1:]))[None]
    pr = P.with_state(pr, w0, viscous=False, sensor_mode=P.SENSOR_OFF, central_order=2 * L)
    c = oracle.rhs(pr, terms=oracle.T_CONV)
    u = w0[1:4] / w0[0]
    dk = (u * c[1:4]).sum(axis=0) - 0.5 * (u * u).sum(axis=0) * c[0]
    scale = np.abs((u * c[1:4]).sum(axis=0)).sum()
    assert abs(dk.sum()) < 1e-13 * scale and scale > 1.0


@pytest.mark.parametrize("central,weno", [(2, 3), (6, 7), (6, 5), (2, 7)])
@pytest.mark.parametrize("mode", [P.SENSOR_HYBRID, P.SENSOR_WENO_ALL])
def test_periodic_conservation_for_every_order(central, weno, mode):
    pr = P.decaying_turbulence(16, mach=1.5, re=500.0, seed=5)
    pr = P.with_state(pr, pr.w0, viscous=False, sensor_mode=mode, theta_star=0.05,
                      central_order=central, weno_order=weno)
    r = oracle.rhs(pr)
    for m in range(5):
        scale = np.abs(r[m]).max() * r[m].size
        assert abs(r[m].sum()) < 1e-13 * scale, (m, r[m].sum(), scale)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_interface_flags_cover_the_central_stencil(L):
    """Interface i+1/2 is shock-capturing iff a node among i-L+1..i+L is
    flagged (periodic box, brute force from the node flags)."""
    pr = P.decaying_turbulence(16, mach=1.5, re=500.0, seed=9)
    pr = P.with_state(pr, pr.w0, viscous=False, sensor_mode=P.SENSOR_HYBRID, theta_star=0.3,
                      central_order=2 * L)
    _, _, nfl, ifl, _ = oracle.rhs(pr, want_flags=True)
    assert 0 < nfl.sum() < nfl.size // 2
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        expect = np.zeros_like(nfl)
        for o in range(1 - L, L + 1):
            expect |= np.roll(nfl, -o, ax)
        assert np.array_equal((ifl >> d) & 1, expect), (L, d)


@pytest.mark.parametrize("weno", [3, 7])
def test_sod_shock_tube_against_exact_riemann_for_weno_orders(weno, monkeypatch):
    """The shock-capturing flux with WENO3 and WENO7 converges to the exact
    Riemann solution and puts the shock within two cells."""
    orig = P.sod_tube

    def sod(n, axis=0, **kw):
        pr = orig(n, axis=axis, **kw)
        return P.with_state(pr, pr.w0, weno_order=weno)

    monkeypatch.setattr(P, "sod_tube", sod)
    errs = []
    for n in (100, 200):
        s, rho, ex, _ = _sod_run(n, 0)
        errs.append(np.mean(np.abs(rho - ex)) * 2.0)
    assert errs[1] < errs[0] and errs[1] < (0.03 if weno == 3 else 0.02), errs
    ps, us = exact.riemann_star(P.SOD_LEFT, P.SOD_RIGHT)
    rs = 0.125 * (ps / 0.1 + 1 / 6) / (ps / 0.1 / 6 + 1)
    xs = 1.0 + us * rs / (rs - 0.125) * 0.2
    idx = np.where((s > 1.3) & (s < 1.5) & (rho < 0.5 * (rs + 0.125)))[0][0]
    assert abs(s[idx] - xs) < 2 * (2.0 / 200)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_viscous_time_step_uses_the_second_derivative_spectral_radius(L):
    """Viscosity-dominated uniform state: dt = CFL 2.5/(rho_2 nu_eff sum h^-2)
    with rho_2 = max over wavenumbers of |symbol of D2| (order 2L, weights
    from the Taylor system)."""
    b = taylor_weights(L, 2)
    th = np.linspace(0.0, math.pi, 20001)
    sym = float(b[0]) + sum(2.0 * float(b[l]) * np.cos(l * th) for l in range(1, L + 1))
    rho2 = np.abs(sym).max()
    pr = P.taylor_green(8)
    shape = pr.w0.shape[1:]
    rho, p = 1.0, 1.0
    w0 = P.conserved_from_primitive(np.full(shape, rho), np.zeros(shape), np.zeros(shape),
                                    np.zeros(shape), np.full(shape, p), 1.4)
    pr2 = P.with_state(pr, w0, viscous=True, mu_ref=200.0, central_order=2 * L)
    T = p / (rho * pr2.R_gas)
    t = T / pr2.T_ref
    mu = pr2.mu_ref * t ** 1.5 * (1 + pr2.S_suth) / (t + pr2.S_suth)
    h = 2 * math.pi / 8
    vf = max(4.0 / 3.0, pr2.gamma / pr2.Pr)
    dv = 2.5 / (rho2 * vf * (mu / rho) * 3.0 / h ** 2)
    c = math.sqrt(1.4 * p / rho)
    dconv = 1.0 / (3 * c / h)
    assert dv < dconv  # the viscous bound is the active one
    assert abs(oracle.dt(pr2, cfl=0.8) - 0.8 * dv) < 1e-12 * dv


def test_invalid_orders_are_rejected():
    pr = P.taylor_green(8)
    for co, wo in ((8, 5), (4, 9), (3, 5), (4, 4)):
        with pytest.raises(ValueError):
            oracle.rhs(with_orders(pr, central=co, weno=wo))
