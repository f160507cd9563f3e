"""Further pins of the FP64 oracle: the characteristic Lax-Friedrichs WENO
flux (Sec. 2.1), the staggered-wall and imposed-shock ghost nodes (Sec. 3.1,
Sec. 3.3) and the volume totals behind the diagnostics.

Each test checks the oracle against something other than itself: a
special case that reduces to the scalar textbook reconstruction, an exact
property of the splitting, an independent eigenvalue computation, closed
forms of the ghost states, an equivalent periodic domain, or plain sums.
"""
import math

import numpy as np
import pytest

import oracle
import problems as P
from tests.test_oracle_pins import _manufactured_problem, _weno5_from_polynomials

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def setup_module(module):
    oracle.build(force=False)


def _line_problem(prim, axis, n, nthin=6, gamma=1.4, weno_order=5):
    """Periodic box, n nodes along `axis` carrying the 1-D primitive fields
    prim = (rho, u, v, w, p) (arrays of length n), uniform across."""
    dims = [nthin, nthin, nthin]
    dims[axis] = n
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    sl = [None, None, None]
    sl[2 - axis] = slice(None)
    f = [np.broadcast_to(np.asarray(a, float)[tuple(sl)], shape).copy() for a in prim]
    w0 = P.conserved_from_primitive(*f, gamma)
    lens = [1.0, 1.0, 1.0]
    lens[axis] = float(n) / nthin
    y, ye, yee = P.uniform_periodic_y(ny, lens[1])
    return P.Problem(name="line", nx=nx, ny=ny, nz=nz, lx=lens[0], lz=lens[2], y=y, y_eta=ye,
                     y_etaeta=yee, gamma=gamma, R_gas=1.0, mu_ref=0.0, viscous=False,
                     sensor_mode=P.SENSOR_WENO_ALL, forcing=False, bcs=P._periodic_bcs(),
                     w0=w0, weno_order=weno_order)


def _line(a, axis):
    """The 1-D line of a (5, nz, ny, nx) array along `axis` at the origin."""
    idx = [0, 0, 0]
    idx[2 - axis] = slice(None)
    return a[(slice(None),) + tuple(idx)]


# ------------------------------------------------------- characteristic WENO
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_entropy_wave_reduces_to_scalar_weno5(axis, sign):
    """Only rho varies (u and p uniform): the state and flux differences lie
    along the entropy eigenvector, the acoustic and shear characteristic
    fields are constant and pass through the splitting unchanged, and the
    entropy field's split flux is u_n rho (plus a constant) upwind.  So the
    mass flux is the scalar WENO5 reconstruction of u_n rho from the upwind
    side, and the other components follow from the affine dependence of the
    exact flux on rho: f = m (1, u, v, w, |u|^2/2) + p (0, e_n, u_n g/(g-1))."""
    n = 40
    rng = np.random.default_rng(11 + axis)
    s = np.arange(n)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * s / n) + 0.1 * rng.uniform(-1, 1, n)
    rho[n // 2:n // 2 + 7] *= 0.35  # a contact discontinuity pair
    vel = np.array([0.4, -0.25, 0.3])
    vel[axis] = sign * 0.7
    p = 0.9
    g = 1.4
    pr = _line_problem([rho, np.full(n, vel[0]), np.full(n, vel[1]), np.full(n, vel[2]),
                        np.full(n, p)], axis, n)
    f = _line(oracle.iface_flux(pr, axis), axis)  # interface i+1/2 at index i
    un = vel[axis]
    m_vals = un * rho
    amp = np.array([1.0, *vel, 0.5 * vel @ vel])
    const = np.zeros(5)
    const[1 + axis] = p
    const[4] = un * p * g / (g - 1)
    for i in range(n):
        if un > 0:
            v5 = m_vals[[(i + o) % n for o in (-2, -1, 0, 1, 2)]]
        else:
            v5 = m_vals[[(i + o) % n for o in (3, 2, 1, 0, -1)]]
        mhat = _weno5_from_polynomials(v5)
        ref = mhat * amp + const
        assert np.abs(f[:, i] - ref).max() <= 1e-12 * np.abs(ref).max(), (i, f[:, i], ref)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stationary_contact_is_kept_exactly(axis):
    """u_n = 0, uniform p, a density jump: the splitting constant of the
    entropy field is max |u_n| = 0, so no dissipation acts on it and the
    mass and energy fluxes vanish at every interface; the momentum flux is
    the pressure (a splitting constant taken from u_n +- c would diffuse the
    contact)."""
    n = 32
    rho = np.where(np.arange(n) < n // 2, 1.0, 0.125)
    vel = np.array([0.3, -0.2, 0.5])
    vel[axis] = 0.0
    pr = _line_problem([rho, np.full(n, vel[0]), np.full(n, vel[1]), np.full(n, vel[2]),
                        np.full(n, 1.0)], axis, n)
    f = _line(oracle.iface_flux(pr, axis), axis)
    assert np.abs(f[0]).max() < 1e-14
    assert np.abs(f[4]).max() < 1e-14
    assert np.abs(f[1 + axis] - 1.0).max() < 1e-14
    for t in range(3):
        if t != axis:
            assert np.abs(f[1 + t]).max() < 1e-14


@pytest.mark.parametrize("weno_order,min_order", [(5, 4.5), (7, 5.5)])
def test_weno_everywhere_design_order_on_smooth_field(weno_order, min_order):
    """Shock-capturing flux at every interface of a smooth 3-D periodic field:
    the inviscid right-hand side converges to the exact divergence-form one
    at the design order (WENO3 is not included: its Jiang-Shu weights lose
    accuracy at smooth extrema)."""
    errs = []
    for n in (16, 32, 64):
        pr, ex_e, _ = _manufactured_problem(n, viscous=False)
        pr = P.with_state(pr, pr.w0, sensor_mode=P.SENSOR_WENO_ALL, weno_order=weno_order)
        r = oracle.rhs(pr, terms=oracle.T_CONV | oracle.T_PRES)
        errs.append([np.abs(r[m] - ex_e[m]).max() / np.abs(ex_e[m]).max() for m in range(5)])
    errs = np.array(errs)
    order = np.log2(errs[-2] / errs[-1])
    assert (order >= min_order).all(), (errs, order)


def _flux_jacobian_eigs(q, d, g):
    """Eigenvalues of the Euler flux Jacobian at conserved state q along d,
    from central differences of the continuous flux (numpy eigvals)."""
    def flux(wv):
        rho = wv[0]
        u = wv[1:4] / rho
        p = (g - 1) * (wv[4] - 0.5 * rho * u @ u)
        f = np.zeros(5)
        f[0] = rho * u[d]
        f[1:4] = rho * u[d] * u
        f[1 + d] += p
        f[4] = u[d] * (wv[4] + p)
        return f
    J = np.zeros((5, 5))
    for k in range(5):
        e = np.zeros(5)
        e[k] = 1e-6 * max(1.0, abs(q[k]))
        J[:, k] = (flux(q + e) - flux(q - e)) / (2 * e[k])
    return np.sort(np.linalg.eigvals(J).real)


@pytest.mark.parametrize("weno_order", [3, 5, 7])
def test_splitting_constants_are_stencil_maxima(weno_order):
    """The Lax-Friedrichs constant of each characteristic field is the largest
    |eigenvalue| of that field over the 2r stencil nodes i-r+1..i+r, checked
    against eigenvalues of the flux Jacobian computed independently."""
    r = (weno_order + 1) // 2
    n = 12
    pr = P.with_state(P.taylor_green(n), P.random_state(n, n, n, seed=3, amp=0.3, mach=1.2),
                      sensor_mode=P.SENSOR_WENO_ALL, weno_order=weno_order)
    w0 = pr.w0
    rng = np.random.default_rng(weno_order)
    for _ in range(6):
        d = int(rng.integers(0, 3))
        i, j, k = (int(x) for x in rng.integers(0, n, 3))
        a = oracle.lf_alpha(pr, d, i, j, k)
        eigs = []
        for t in range(-r + 1, r + 1):
            idx = [i, j, k]
            idx[d] = (idx[d] + t) % n
            eigs.append(_flux_jacobian_eigs(w0[:, idx[2], idx[1], idx[0]], d, pr.gamma))
        eigs = np.abs(np.array(eigs))  # per node, ascending: u-c, u, u, u, u+c
        ref = np.array([eigs[:, 0].max(), eigs[:, 2].max(), eigs[:, 2].max(), eigs[:, 2].max(),
                        eigs[:, 4].max()])
        assert np.abs(a - ref).max() <= 1e-7 * ref.max(), (a, ref)
        # the stencil is not uniform: a range one node short would differ
        assert np.ptp(eigs[:, 4]) > 1e-3


@pytest.mark.parametrize("weno_order", [3, 5, 7])
def test_weno_flux_reads_exactly_its_stencil(weno_order):
    """The flux at i+1/2 changes when any of the 2r nodes i-r+1..i+r changes
    and is bitwise unchanged when a node outside them changes."""
    r = (weno_order + 1) // 2
    n = 16
    axis = 0
    rng = np.random.default_rng(5)
    rho = 1 + 0.4 * rng.uniform(-1, 1, n)
    u = 0.6 * rng.uniform(-1, 1, n)
    p = 1 + 0.4 * rng.uniform(-1, 1, n)
    z = np.zeros(n)
    base = _line_problem([rho, u, z, z, p], axis, n, weno_order=weno_order)
    i = 7
    f0 = _line(oracle.iface_flux(base, axis), axis)[:, i]
    for t in range(i - r - 2, i + r + 3):
        rho2 = rho.copy()
        rho2[t % n] *= 1.05
        pr = _line_problem([rho2, u, z, z, p], axis, n, weno_order=weno_order)
        f1 = _line(oracle.iface_flux(pr, axis), axis)[:, i]
        inside = i - r + 1 <= t <= i + r
        if inside:
            assert np.abs(f1 - f0).max() > 1e-9, t
        else:
            assert np.array_equal(f1, f0), t


# ------------------------------------------------------- ghost nodes (Sec. 3.1, 3.3)
def _wall_problem(kind, nx=10, ny=12, nz=6, seed=4, T_w=1.3):
    rng = np.random.default_rng(seed)
    y, ye, yee = P.uniform_periodic_y(ny, 2.0)
    y = y + 1.0 / ny
    shape = (nz, ny, nx)
    X = np.arange(nx)[None, None, :] * (2 * np.pi / nx)
    Yc = (np.arange(ny)[None, :, None] + 0.5) / ny
    Zc = np.arange(nz)[:, None, None] * (2 * np.pi / nz)
    rho = 1 + 0.2 * np.sin(X + 2 * Zc) * np.cos(3 * Yc) + 0.02 * rng.uniform(-1, 1, shape)
    u = 0.5 * np.sin(np.pi * Yc) + 0.1 * np.cos(X - Zc)
    v = 0.2 * np.sin(2 * np.pi * Yc) * np.cos(X)
    w = 0.15 * np.cos(2 * Zc + Yc)
    T = 1 + 0.25 * np.cos(2 * np.pi * Yc + X)
    g, Rg = 1.4, 1.0 / (1.4 * 0.8 ** 2)
    p = rho * Rg * T
    w0 = P.conserved_from_primitive(rho, u, v, w, p, g)
    params = np.array([T_w]) if kind == P.BC_WALL_ISOTHERMAL else np.zeros(0)
    bcs = P._periodic_bcs()
    bcs[P.FACE_YM] = (kind, params)
    bcs[P.FACE_YP] = (kind, params)
    return P.Problem(name="walls", nx=nx, ny=ny, nz=nz, lx=2 * np.pi, lz=2 * np.pi, y=y,
                     y_eta=ye, y_etaeta=yee, gamma=g, R_gas=Rg, mu_ref=0.02, T_ref=1.0,
                     S_suth=0.368, viscous=True, sensor_mode=P.SENSOR_OFF, forcing=False,
                     bcs=bcs, w0=w0)


def _prims(w, g, Rg):
    rho = w[0]
    u, v, ww = w[1] / rho, w[2] / rho, w[3] / rho
    p = (g - 1) * (w[4] - 0.5 * rho * (u * u + v * v + ww * ww))
    return rho, u, v, ww, p, p / (rho * Rg)


@pytest.mark.parametrize("kind", [P.BC_WALL_ADIABATIC, P.BC_WALL_ISOTHERMAL])
def test_staggered_wall_ghosts_closed_form(kind):
    """Ghost s mirrors node s-1 across the wall half-way between node 0 and
    ghost 1: velocity reversed, pressure kept, temperature kept (adiabatic)
    or reflected about T_w (isothermal), density from the gas law.  Hence
    the linear interpolation to the wall gives u = 0 and, for the isothermal
    wall, T = T_w; for the adiabatic wall the temperature is even about the
    wall (zero wall-normal gradient, no heat flux through it)."""
    T_w = 1.3
    pr = _wall_problem(kind, T_w=T_w)
    g, Rg = pr.gamma, pr.R_gas
    w0 = pr.w0
    for face in (2, 3):
        gh = oracle.ghosts_y(pr, face)
        hw = gh.shape[1]
        for s in range(1, hw + 1):
            j_m = s - 1 if face == 2 else pr.ny - s
            mirror = w0[:, :, j_m, :]                  # (5, nz, nx)
            ghost = gh[:, s - 1, :, hw:hw + pr.nx]      # interior x range
            rm, um, vm, wm, pm, Tm = _prims(mirror, g, Rg)
            rg, ug, vg, wg, pg, Tg = _prims(ghost, g, Rg)
            tol = 1e-13
            assert np.abs(ug + um).max() < tol and np.abs(vg + vm).max() < tol
            assert np.abs(wg + wm).max() < tol
            assert np.abs(pg - pm).max() < tol * np.abs(pm).max()
            if kind == P.BC_WALL_ADIABATIC:
                assert np.abs(Tg - Tm).max() < tol
                # conserved ghost = (rho, -rho u, -rho v, -rho w, rho E) of the mirror
                ref = mirror * np.array([1, -1, -1, -1, 1])[:, None, None]
                assert np.abs(ghost - ref).max() < 1e-13 * np.abs(ref).max()
            else:
                assert np.abs(0.5 * (Tg + Tm) - T_w).max() < tol
                assert np.abs(rg - pm / (Rg * (2 * T_w - Tm))).max() < tol


@pytest.mark.parametrize("kind", [P.BC_WALL_ADIABATIC, P.BC_WALL_ISOTHERMAL])
def test_walls_equal_their_mirrored_periodic_domain(kind):
    """A channel between two staggered walls equals, for every term that uses
    the ghosts the same way, the periodic domain of twice the height that
    holds the field and its mirror image (velocity reversed, temperature
    kept or reflected about T_w): viscous and heat-flux terms and the
    pressure term in all equations, and, for the adiabatic wall, the
    convective mass and energy fluxes (density and enthalpy are then even
    about the wall, so the mirror makes the wall-interface pair sums cancel,
    which is the zero convective wall flux).  Wrong mirror indices, signs or
    temperatures fail it."""
    T_w = 1.3
    pr = _wall_problem(kind, T_w=T_w)
    g, Rg = pr.gamma, pr.R_gas
    rho, u, v, w, p, T = _prims(pr.w0, g, Rg)
    Tm = T if kind == P.BC_WALL_ADIABATIC else 2 * T_w - T
    rm = p / (Rg * Tm)
    mir = P.conserved_from_primitive(rm, -u, -v, -w, p, g)[:, :, ::-1, :]
    ny = pr.ny
    wd = np.concatenate([mir, pr.w0], axis=2)       # rows: mirror (reversed), then field
    y, ye, yee = P.uniform_periodic_y(2 * ny, 4.0)
    dbl = P.Problem(name="doubled", nx=pr.nx, ny=2 * ny, nz=pr.nz, lx=pr.lx, lz=pr.lz, y=y,
                    y_eta=ye, y_etaeta=yee, gamma=g, R_gas=Rg, mu_ref=pr.mu_ref, T_ref=1.0,
                    S_suth=pr.S_suth, viscous=True, sensor_mode=P.SENSOR_OFF, forcing=False,
                    bcs=P._periodic_bcs(), w0=wd)
    checks = [(oracle.T_VISC | oracle.T_PRES, range(5))]
    if kind == P.BC_WALL_ADIABATIC:  # even density and enthalpy: the pair sums cancel
        checks.append((oracle.T_CONV, (0, 4)))
    for terms, comps in checks:
        r_wall = oracle.rhs(pr, terms=terms)
        r_dbl = oracle.rhs(dbl, terms=terms)[:, :, ny:, :]
        for m in comps:
            scale = max(np.abs(r_wall[m]).max(), 1e-300)
            assert np.abs(r_wall[m] - r_dbl[m]).max() <= 1e-12 * scale, (terms, m)
    assert np.abs(oracle.rhs(pr, terms=oracle.T_VISC)[4]).max() > 1e-3  # non-trivial


def test_shock_top_ghosts_take_the_two_states():
    """Imposed oblique shock (Sec. 3.3): ghost nodes of the top face hold the
    free-stream state for i < i_shock and the post-shock state from i_shock
    on, over the whole x-extended range."""
    pr = P.small_sbli(48, 16, 6)
    kind, params = pr.bcs[P.FACE_YP]
    assert kind == P.BC_SHOCK_TOP
    ish = int(params[0])
    assert 0 < ish < pr.nx
    s1 = P.conserved_from_primitive(*params[1:6], pr.gamma)
    s2 = P.conserved_from_primitive(*params[6:11], pr.gamma)
    gh = oracle.ghosts_y(pr, 3)
    hw = gh.shape[1]
    i = np.arange(-hw, pr.nx + hw)
    for m in range(5):
        ref = np.where(i < ish, s1[m], s2[m])
        assert np.abs(gh[m] - ref[None, None, :]).max() <= 1e-14 * abs(ref).max()
    # the two states differ, so the test sees the switch position
    assert np.abs(s1 - s2).max() > 0.1 * np.abs(s1).max()


# ------------------------------------------------------- totals
def test_totals_are_volume_sums():
    """Mass, momentum, total and kinetic energy as plain volume sums with
    dV = dx dz d_eta y_eta (stretched walls)."""
    pr = P.small_channel(24, 20, 12)
    w = pr.w0
    dv = pr.dx * pr.dz * (1.0 / pr.ny) * pr.y_eta[None, :, None]
    ref = [np.sum(w[m] * dv) for m in range(5)]
    ref.append(np.sum(0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / w[0] * dv))
    tot = oracle.totals(pr, w)
    assert np.abs(tot - np.array(ref)).max() <= 1e-12 * np.abs(ref).max()
    assert abs(tot[0] - np.sum(w[0] * dv)) <= 1e-13 * tot[0]


def test_extrema_closed_form():
    """Minimum density and pressure and maximum Mach number of a field whose
    extrema sit at known nodes with known values: rho = 1 + 0.4 cos(x)
    cos(y) cos(z) reaches 0.6 at the node (pi, 0, 0), p = (1 - 0.3 sin^2 ...)
    / gamma, and a single node moves at u = 2.5 c where everything else is
    subsonic; non-finite conserved values are counted one by one and kept
    out of the extrema."""
    g = 1.4
    n = 16
    pr = P.taylor_green(n)
    x = np.arange(n) * (2 * np.pi / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho = 1.0 + 0.4 * np.cos(X) * np.cos(Y) * np.cos(Z)
    p = (1.0 - 0.3 * np.sin(X) ** 2 * np.sin(Z) ** 2) / g   # min 0.7/g at sin = +-1
    c = np.sqrt(g * p / rho)
    u = 0.2 * c * np.sin(Y)
    v = np.zeros_like(u)
    ww = np.zeros_like(u)
    u[3, 5, 7] = 2.5 * c[3, 5, 7]
    w = P.conserved_from_primitive(rho, u, v, ww, p, pr.gamma)
    assert pr.gamma == g
    ex = oracle.extrema(pr, w)
    assert abs(ex[0] - 0.6) <= 1e-15
    assert abs(ex[1] - 0.7 / g) <= 1e-15
    assert abs(ex[2] - 2.5) <= 1e-13
    assert ex[3] == 0
    # poison two points: three non-finite values, the extrema unchanged
    w2 = w.copy()
    w2[0, 8, 0, 0] = 0.1           # a low density at a point whose energy is infinite
    w2[4, 8, 0, 0] = np.inf
    w2[2, 1, 1, 1] = -np.inf
    w2[3, 1, 1, 1] = np.nan
    ex2 = oracle.extrema(pr, w2)
    assert ex2[3] == 3
    assert abs(ex2[0] - 0.6) <= 1e-15 and abs(ex2[1] - 0.7 / g) <= 1e-15 and abs(ex2[2] - 2.5) <= 1e-13


def test_boundary_layer_wall_is_a_reflecting_recovery_temperature_wall():
    """The boundary-layer wall (Sec. 3.2: characteristic treatment at the
    no-slip wall with the temperature at its nominal recovery value T_r =
    1 + (gamma-1)/2 Pr^(1/3) M^2) is the staggered isothermal wall at T_r.
    Linearised about the wall state with any impedance Z = rho c, the
    acoustic invariant entering the domain from each ghost equals the one
    leaving through the wall from its mirror node, p_g + Z v_g = p_m - Z v_m
    (total reflection of the outgoing wave, as the characteristic wall
    condition of zero normal velocity prescribes), the tangential velocity
    and the temperature interpolate to 0 and T_r at the wall, and the ghost
    pressure equals the mirror's (no pressure gradient forced through the
    wall)."""
    pr = P.small_boundary_layer()
    kind, params = pr.bcs[P.FACE_YM]
    M = 2.0
    T_r = 1.0 + 0.5 * (pr.gamma - 1.0) * pr.Pr ** (1.0 / 3.0) * M * M
    assert kind == P.BC_WALL_ISOTHERMAL and abs(params[0] - T_r) <= 1e-15 * T_r
    rng = np.random.Generator(np.random.PCG64(3))
    w0 = pr.w0.copy()
    w0[2] += 0.05 * rng.uniform(-1, 1, w0[2].shape) * w0[0]   # wall-normal motion to reflect
    prw = P.with_state(pr, w0)
    g, Rg = pr.gamma, pr.R_gas
    gh = oracle.ghosts_y(prw, 2)
    hw = gh.shape[1]
    for s in range(1, hw + 1):
        mirror = w0[:, :, s - 1, :]
        ghost = gh[:, s - 1, :, hw:hw + pr.nx]
        rm, um, vm, wm, pm, Tm = _prims(mirror, g, Rg)
        rg, ug, vg, wg, pg, Tg = _prims(ghost, g, Rg)
        for Z in (0.5, 1.0, float(np.sqrt(g * pm.mean() / rm.mean()) * rm.mean())):
            w_in = pg + Z * vg
            w_out = pm - Z * vm
            assert np.abs(w_in - w_out).max() <= 1e-13 * np.abs(pm).max()
        assert np.abs(0.5 * (ug + um)).max() <= 1e-15 and np.abs(0.5 * (wg + wm)).max() <= 1e-15
        assert np.abs(0.5 * (Tg + Tm) - T_r).max() <= 1e-13 * T_r
        assert np.abs(pg - pm).max() <= 1e-13 * np.abs(pm).max()
    assert np.abs(w0[2][:, 0, :]).max() > 1e-3  # the reflected wave is not trivial
