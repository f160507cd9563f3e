"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This package builds *inputs only*: grids (node coordinates and the analytic
metric of the wall-normal mapping), physical parameters, boundary-condition
descriptors and initial conserved-variable arrays.  It performs none of the
discretisation (no fluxes, derivatives, sensor, time stepping or
reductions); both the oracle and the GPU library receive the arrays built
here and compute everything else on their own.

Conventions (non-dimensionalisation; the paper does not state one, Sec. 2):
reference density, velocity, temperature and length are 1, the gas constant
is R = 1/(gamma M_r^2) so that the reference sound speed is 1/M_r,
c_v = R/(gamma-1), c_p = gamma R/(gamma-1) and mu(T_ref) = mu_ref.

Array layout: conserved variables w[5][nz][ny][nx] (float64, x fastest),
w = (rho, rho u, rho v, rho w, rho E) as in Sec. 2.2.

Grid: x and z are uniform, dx = lx/nx, x_i = i dx (likewise z).  The y
direction is described on a computational coordinate eta with d_eta = 1/ny
and the analytic metric y_eta = dy/deta, y_etaeta = d2y/deta2 at each node;
a uniform periodic y has y_eta = ly and y_etaeta = 0.  With walls the nodes
sit at eta_j = (j + 1/2)/ny so that the walls fall on the intermediate
nodes eta = 0 and 1 (staggered wall, Sec. 3.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------- BC kinds
BC_PERIODIC = 0
BC_WALL_ISOTHERMAL = 1   # params: [T_wall]
BC_WALL_ADIABATIC = 2    # params: []
BC_DIRICHLET = 3         # params: primitives (rho,u,v,w,p) per transverse j, shape (5, ny)
BC_OUTFLOW_CHAR = 4      # params: []
BC_SHOCK_TOP = 5         # params: [i_shock, rho1,u1,v1,w1,p1, rho2,u2,v2,w2,p2]
BC_DF_INFLOW = 6         # params: see df_inflow_params (x- face only)

FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = range(6)

SENSOR_OFF, SENSOR_HYBRID, SENSOR_WENO_ALL = 0, 1, 2

BASE_SEED = 20040227


@dataclasses.dataclass
class Problem:
    """Everything needed to evaluate the right-hand side and to step."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    y: np.ndarray            # (ny,) node coordinates (informational)
    y_eta: np.ndarray        # (ny,) dy/deta at nodes, deta = 1/ny
    y_etaeta: np.ndarray     # (ny,) d2y/deta2 at nodes
    gamma: float = 1.4
    Pr: float = 0.72
    R_gas: float = 1.0
    mu_ref: float = 0.0
    T_ref: float = 1.0
    S_suth: float = 110.4 / 300.0
    viscous: bool = True
    sensor_mode: int = SENSOR_OFF
    theta_star: float = 0.1
    sensor_eps: float = 1.0
    forcing: bool = False
    bcs: List[Tuple[int, np.ndarray]] = dataclasses.field(
        default_factory=lambda: [(BC_PERIODIC, np.zeros(0))] * 6)
    w0: Optional[np.ndarray] = None   # (5, nz, ny, nx)
    cfl: float = 0.8
    nsteps: int = 10
    central_order: int = 4   # order 2L of the central flux and viscous terms: 2, 4 or 6
    weno_order: int = 5      # order 2r-1 of the WENO reconstruction: 3, 5 or 7

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dz(self) -> float:
        return self.lz / self.nz

    def x(self) -> np.ndarray:
        return np.arange(self.nx) * self.dx

    def z(self) -> np.ndarray:
        return np.arange(self.nz) * self.dz


# ------------------------------------------------------------------ grids
def uniform_periodic_y(ny: int, ly: float):
    y = np.arange(ny) * (ly / ny)
    return y, np.full(ny, float(ly)), np.zeros(ny)


def tanh_channel_y(ny: int, beta: float = 2.0):
    """Wall-clustered channel map y = tanh(beta(2 eta - 1))/tanh(beta), y in [-1, 1]."""
    eta = (np.arange(ny) + 0.5) / ny
    a = beta * (2.0 * eta - 1.0)
    th = math.tanh(beta)
    t = np.tanh(a)
    sech2 = 1.0 - t * t
    y = t / th
    y_eta = 2.0 * beta * sech2 / th
    y_etaeta = -8.0 * beta * beta * sech2 * t / th
    return y, y_eta, y_etaeta


def sinh_wall_y(ny: int, ly: float, beta: float = 2.5):
    """Wall-clustered boundary-layer map y = ly sinh(beta eta)/sinh(beta), wall at y = 0."""
    eta = (np.arange(ny) + 0.5) / ny
    sb = math.sinh(beta)
    y = ly * np.sinh(beta * eta) / sb
    y_eta = ly * beta * np.cosh(beta * eta) / sb
    y_etaeta = ly * beta * beta * np.sinh(beta * eta) / sb
    return y, y_eta, y_etaeta


def periodic_stretched_y(ny: int, ly: float, amp: float = 0.3):
    """Smooth periodic stretching y = ly (eta + amp sin(2 pi eta)/(2 pi)), eta_j = j/ny.

    Used by tests to exercise the metric terms without walls."""
    eta = np.arange(ny) / ny
    tp = 2.0 * math.pi
    y = ly * (eta + amp * np.sin(tp * eta) / tp)
    y_eta = ly * (1.0 + amp * np.cos(tp * eta))
    y_etaeta = -ly * amp * tp * np.sin(tp * eta)
    return y, y_eta, y_etaeta


# ------------------------------------------------------- thermodynamics in
def conserved_from_primitive(rho, u, v, w, p, gamma):
    """(rho,u,v,w,p) -> (rho, rho u, rho v, rho w, rho E) with E = c_v T + |u|^2/2."""
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, e]).astype(np.float64)


def sutherland_S(T_ref_dim: float) -> float:
    """Sutherland constant 110.4 K made non-dimensional by the reference temperature."""
    return 110.4 / T_ref_dim


def _rng(cfg_index: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + cfg_index + 1000 * extra))


def _periodic_bcs():
    return [(BC_PERIODIC, np.zeros(0)) for _ in range(6)]


# -------------------------------------------------------- Taylor-Green vortex
def taylor_green(n: int = 32, mach: float = 0.1, re: float = 1600.0,
                 noise: float = 1e-6, seed_index: int = 0) -> Problem:
    """3-D periodic Taylor-Green vortex on [0, 2pi)^3 with seeded density noise."""
    g = 1.4
    R = 1.0 / (g * mach * mach)
    L = 2.0 * math.pi
    y, ye, yee = uniform_periodic_y(n, L)
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p0 = R  # rho0 = T0 = 1
    p = p0 + (1.0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = p / (R * 1.0)
    xi = _rng(seed_index).uniform(-1.0, 1.0, size=rho.shape)
    rho = rho * (1.0 + noise * xi)
    w0 = conserved_from_primitive(rho, u, v, w, p, g)
    return Problem(name=f"tgv{n}", nx=n, ny=n, nz=n, lx=L, lz=L, y=y, y_eta=ye,
                   y_etaeta=yee, gamma=g, Pr=0.72, R_gas=R, mu_ref=1.0 / re, T_ref=1.0,
                   S_suth=sutherland_S(300.0), viscous=True, sensor_mode=SENSOR_OFF,
                   theta_star=0.1, sensor_eps=1.0, forcing=False, bcs=_periodic_bcs(),
                   w0=w0, cfl=0.8, nsteps=10)


# ------------------------------------------------------------ channel flow
def channel(nx: int = 256, ny: int = 128, nz: int = 128, mach_b: float = 1.5,
            re_b: float = 3000.0, noise: float = 0.1, seed_index: int = 1,
            sensor_mode: int = SENSOR_HYBRID, theta_star: float = 0.1,
            beta: float = 2.0, nsteps: int = 100) -> Problem:
    """Compressible channel between isothermal walls at y = -1, 1 (half height h = 1).

    Laminar compressible Poiseuille start: u = U(1 - y^2), the constant-mu
    laminar energy balance T = 1 + (Pr (gamma-1) M_b^2 U^2/3)(1 - y^4) with
    U = 3/2, a uniform pressure giving unit bulk density, U rescaled to unit
    bulk momentum, then seeded uniform velocity noise of amplitude `noise`.
    Bulk Reynolds number uses the full height: Re_b = 2 rho_b u_b h / mu_w."""
    g, Pr = 1.4, 0.72
    R = 1.0 / (g * mach_b * mach_b)
    lx, lz = 6.0 * math.pi, 2.0 * math.pi
    y, ye, yee = tanh_channel_y(ny, beta)
    wgt = ye  # nodal volume weights (uniform x,z)
    Ucl = 1.5
    T1 = 1.0 + (Pr * (g - 1.0) * mach_b ** 2 * Ucl ** 2 / 3.0) * (1.0 - y ** 4)
    p = R / (np.sum(wgt / T1) / np.sum(wgt))
    rho1 = p / (R * T1)
    u1 = Ucl * (1.0 - y * y)
    scale = np.sum(rho1 * u1 * wgt) / np.sum(wgt)
    u1 = u1 / scale
    shape = (nz, ny, nx)
    rho = np.broadcast_to(rho1[None, :, None], shape).copy()
    pp = np.full(shape, p)
    u = np.broadcast_to(u1[None, :, None], shape).copy()
    rng = _rng(seed_index)
    xi = rng.uniform(-1.0, 1.0, size=(3,) + shape)
    u = u + noise * xi[0]
    v = noise * xi[1]
    w = noise * xi[2]
    w0 = conserved_from_primitive(rho, u, v, w, pp, g)
    mu_w = 2.0 / re_b
    bcs = _periodic_bcs()
    bcs[FACE_YM] = (BC_WALL_ISOTHERMAL, np.array([1.0]))
    bcs[FACE_YP] = (BC_WALL_ISOTHERMAL, np.array([1.0]))
    return Problem(name=f"channel{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, lx=lx, lz=lz,
                   y=y, y_eta=ye, y_etaeta=yee, gamma=g, Pr=Pr, R_gas=R, mu_ref=mu_w,
                   T_ref=1.0, S_suth=sutherland_S(300.0), viscous=True,
                   sensor_mode=sensor_mode, theta_star=theta_star, sensor_eps=1.0,
                   forcing=True, bcs=bcs, w0=w0, cfl=0.8, nsteps=nsteps)


# ------------------------------------------------------------ oblique shock
def oblique_shock(mach: float, deflection_deg: float, gamma: float = 1.4):
    """Weak-branch oblique shock: wave angle beta and jump ratios.

    Solves tan(delta) = 2 cot(beta) (M^2 sin^2 beta - 1)/(M^2 (gamma + cos 2beta) + 2)
    by bisection on the weak branch, then applies the normal-shock
    Rankine-Hugoniot relations to M_n = M sin(beta).  Returns
    (beta_rad, p2/p1, rho2/rho1, M2)."""
    d = math.radians(deflection_deg)

    def f(b):
        return (2.0 / math.tan(b) * (mach ** 2 * math.sin(b) ** 2 - 1.0)
                / (mach ** 2 * (gamma + math.cos(2.0 * b)) + 2.0) - math.tan(d))

    lo = math.asin(1.0 / mach) + 1e-12
    # the deflection is maximal near beta_max; bracket the weak root below it
    bs = np.linspace(lo, math.pi / 2 - 1e-9, 20001)
    vals = np.array([f(b) for b in bs])
    idx = int(np.argmax(vals > 0))
    a, b = bs[idx - 1], bs[idx]
    for _ in range(200):
        m = 0.5 * (a + b)
        if f(a) * f(m) <= 0:
            b = m
        else:
            a = m
    beta = 0.5 * (a + b)
    mn1 = mach * math.sin(beta)
    p21 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (mn1 ** 2 - 1.0)
    r21 = (gamma + 1.0) * mn1 ** 2 / ((gamma - 1.0) * mn1 ** 2 + 2.0)
    mn2 = math.sqrt((1.0 + 0.5 * (gamma - 1.0) * mn1 ** 2)
                    / (gamma * mn1 ** 2 - 0.5 * (gamma - 1.0)))
    m2 = mn2 / math.sin(beta - d)
    return beta, p21, r21, m2


# ---------------------------------------------------- shock/boundary-layer box
# Node-flag threshold for the shock/boundary-layer box at 1024x256x128,
# chosen by hand so that about 5% of the nodes are flagged on the initial
# field (the 95th percentile of the sensor there is 0.156); a CPU test checks
# the fraction with the oracle.
SBLI_THETA_STAR = 0.155


def sbli(nx: int = 1024, ny: int = 256, nz: int = 128, mach: float = 2.0,
         re_delta: float = 2000.0, deflection_deg: float = 8.0, noise: float = 0.05,
         seed_index: int = 2, theta_star: Optional[float] = None,
         nsteps: int = 200) -> Problem:
    """Oblique shock impinging on a laminar boundary layer over an adiabatic wall.

    Box 4 x 1 x 0.5, inflow boundary-layer thickness delta_in = 1/20 of the
    height, u = tanh(2.6467 y/delta_in), recovery-form temperature
    T = 1 + r (gamma-1)/2 M^2 (1 - u^2) with r = Pr^(1/3), uniform pressure,
    seeded velocity noise inside the layer.  Boundaries: x- Dirichlet (the
    inflow profile), x+ characteristic outflow, y- adiabatic wall, y+ the
    free stream upstream of the shock foot and the post-shock state
    downstream of it (x_sh = x_imp - L_y/tan(beta), x_imp = 2.5), z periodic."""
    g, Pr = 1.4, 0.72
    R = 1.0 / (g * mach * mach)
    lx, ly, lz = 4.0, 1.0, 0.5
    delta = ly / 20.0
    y, ye, yee = sinh_wall_y(ny, ly, 2.5)
    u1 = np.tanh(2.6467 * y / delta)
    r = Pr ** (1.0 / 3.0)
    T1 = 1.0 + r * 0.5 * (g - 1.0) * mach * mach * (1.0 - u1 * u1)
    pinf = R  # rho_inf = T_inf = 1
    rho1 = pinf / (R * T1)
    shape = (nz, ny, nx)
    rho = np.broadcast_to(rho1[None, :, None], shape).copy()
    u = np.broadcast_to(u1[None, :, None], shape).copy()
    rng = _rng(seed_index)
    xi = rng.uniform(-1.0, 1.0, size=(3,) + shape)
    inside = (y < delta)[None, :, None]
    u = u + noise * xi[0] * inside
    v = noise * xi[1] * inside
    w = noise * xi[2] * inside
    pp = np.full(shape, pinf)
    w0 = conserved_from_primitive(rho, u, v, w, pp, g)
    # shock states
    beta, p21, r21, _ = oblique_shock(mach, deflection_deg, g)
    d = math.radians(deflection_deg)
    # velocity behind the shock: tangential component preserved, flow turned towards the wall
    un1 = math.sin(beta)
    ut = math.cos(beta)
    un2 = un1 / r21
    vmag = math.hypot(un2, ut)
    u2 = vmag * math.cos(d)
    v2 = -vmag * math.sin(d)
    x_imp = 2.5
    x_sh = x_imp - ly / math.tan(beta)
    dx = lx / nx
    i_sh = int(math.ceil(x_sh / dx - 1e-12))
    prof = np.stack([rho1, u1, np.zeros(ny), np.zeros(ny), np.full(ny, pinf)])
    bcs = _periodic_bcs()
    bcs[FACE_XM] = (BC_DIRICHLET, prof)
    bcs[FACE_XP] = (BC_OUTFLOW_CHAR, np.zeros(0))
    bcs[FACE_YM] = (BC_WALL_ADIABATIC, np.zeros(0))
    bcs[FACE_YP] = (BC_SHOCK_TOP, np.array([float(i_sh), 1.0, 1.0, 0.0, 0.0, pinf,
                                            r21, u2, v2, 0.0, p21 * pinf]))
    mu_inf = delta / re_delta
    return Problem(name=f"sbli{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, lx=lx, lz=lz,
                   y=y, y_eta=ye, y_etaeta=yee, gamma=g, Pr=Pr, R_gas=R, mu_ref=mu_inf,
                   T_ref=1.0, S_suth=sutherland_S(160.0), viscous=True,
                   sensor_mode=SENSOR_HYBRID,
                   theta_star=SBLI_THETA_STAR if theta_star is None else theta_star,
                   sensor_eps=(1.0 / delta) ** 2, forcing=False, bcs=bcs, w0=w0,
                   cfl=0.8, nsteps=nsteps)


# ----------------------------------------------- spatially developing boundary layer
def musker_uplus(yp):
    """Musker's (1979) explicit inner profile u+(y+) (zero at the wall)."""
    yp = np.asarray(yp, dtype=np.float64)
    return (5.424 * np.arctan((2.0 * yp - 8.15) / 16.7)
            + np.log10((yp + 10.6) ** 9.6 / (yp * yp - 8.15 * yp + 86.0) ** 2)
            - 3.51132976630723)


def bl_vd_uplus(yp, eta, pi_wake: float = 0.45, kappa: float = 0.41):
    """Incompressible (van Driest) profile: Musker inner law plus Coles' wake
    2 Pi/kappa sin^2(pi eta/2), eta = y/delta capped at 1."""
    e = np.minimum(np.asarray(eta, dtype=np.float64), 1.0)
    return musker_uplus(yp) + 2.0 * pi_wake / kappa * np.sin(0.5 * math.pi * e) ** 2


def df_inflow_params(mean_prim: np.ndarray, rstress: np.ndarray, n_y: float, n_z: float,
                     t_lag: float, seed: int) -> np.ndarray:
    """Parameter vector of the digital-filter inflow face: [n_y, n_z (filter
    lengths in grid spacings), T (Lagrangian time scale), seed, mean
    (rho, u, v, w, p)[5][ny], Reynolds stresses (R11, R22, R33, R12, R13,
    R23)[6][ny]].  The filter coefficients and the stress factorisation are
    derived by whoever consumes the vector."""
    head = np.array([float(n_y), float(n_z), float(t_lag), float(seed)])
    return np.concatenate([head, np.asarray(mean_prim, np.float64).ravel(),
                           np.asarray(rstress, np.float64).ravel()])


def boundary_layer(nx: int = 1024, ny: int = 128, nz: int = 128, lx: float = 30.0,
                   ly: float = 12.0, lz: float = 6.0, mach: float = 2.0, re_tau: float = 250.0,
                   beta: float = 3.0, len_y: float = 0.25, len_z: float = 0.25,
                   t_lag: float = 0.5, seed_index: int = 5, theta_star: float = 0.1,
                   nsteps: int = 200) -> Problem:
    """Spatially developing supersonic turbulent boundary layer over an
    isothermal wall at the recovery temperature, lengths in units of the
    inflow thickness delta_in = 1 (free stream: rho = u = T = 1).

    Mean field (Sec. 3.2 recipe): Musker's inner profile with Coles' wake
    as the van Driest velocity, transformed to the compressible profile with
    the Crocco-Busemann temperature for a recovery-temperature wall,
    T(u) = T_r (1 - a^2 u^2), a^2 = (T_r - 1)/T_r, for which the van
    Driest integral inverts in closed form: u = sin(a u_vd)/a.  The friction
    velocity makes u(delta_in) = 0.99; the wall viscosity follows from
    Re_tau.  Inflow: digital filtering with synthetic Reynolds-stress
    profiles (the paper interpolates a DNS database that is not available):
    (R11, R22, R33, R12) = (2.2^2, 1.0^2, 1.4^2, -0.9) u_tau^2 (1 - eta^2)
    (1 - exp(-y+/8))^2 inside the layer, zero outside; filter lengths len_y,
    len_z (in delta_in) and Lagrangian time t_lag.  Outflow and top faces:
    characteristic non-reflecting; spanwise periodic.  The interior starts
    from the mean profile (uniform in x)."""
    g, Pr = 1.4, 0.72
    R = 1.0 / (g * mach * mach)
    Tr = 1.0 + 0.5 * (g - 1.0) * Pr ** (1.0 / 3.0) * mach * mach
    a = math.sqrt((Tr - 1.0) / Tr)
    y, ye, yee = sinh_wall_y(ny, ly, beta)
    eta = y  # delta_in = 1
    uvd_edge = math.asin(0.99 * a) / a
    u_tau = uvd_edge / float(bl_vd_uplus(re_tau, 1.0))
    rho_w = 1.0 / Tr
    mu_w = rho_w * u_tau * 1.0 / re_tau
    yp = y * re_tau
    uvd = u_tau * bl_vd_uplus(yp, eta)
    u = np.where(eta < 1.0, np.sin(np.minimum(a * uvd, 0.5 * math.pi)) / a, 1.0)
    u = np.minimum(u, 1.0)
    T = Tr * (1.0 - a * a * u * u)
    pinf = R  # rho = T = 1 in the free stream
    rho = pinf / (R * T)
    S = sutherland_S(220.0)
    mu_ref = mu_w / (Tr ** 1.5 * (1.0 + S) / (Tr + S))
    # synthetic Reynolds stresses
    damp = (1.0 - np.exp(-yp / 8.0)) ** 2
    h = np.clip(1.0 - eta * eta, 0.0, None) * damp * u_tau * u_tau
    rs = np.stack([2.2 ** 2 * h, 1.0 ** 2 * h, 1.4 ** 2 * h, -0.9 * h, 0.0 * h, 0.0 * h])
    # filter widths in grid spacings (mean spacing inside the layer for y)
    dz = lz / nz
    inside = eta < 1.0
    dy_bl = float(np.mean(np.diff(y[inside]))) if inside.sum() > 1 else float(y[1] - y[0])
    mean = np.stack([rho, u, np.zeros(ny), np.zeros(ny), np.full(ny, pinf)])
    seed = BASE_SEED + seed_index
    params = df_inflow_params(mean, rs, len_y / dy_bl, len_z / dz, t_lag, seed)
    shape = (nz, ny, nx)
    U = np.broadcast_to(u[None, :, None], shape)
    Rh = np.broadcast_to(rho[None, :, None], shape)
    zeros = np.zeros(shape)
    w0 = conserved_from_primitive(Rh, U, zeros, zeros, np.full(shape, pinf), g)
    bcs = _periodic_bcs()
    bcs[FACE_XM] = (BC_DF_INFLOW, params)
    bcs[FACE_XP] = (BC_OUTFLOW_CHAR, np.zeros(0))
    bcs[FACE_YM] = (BC_WALL_ISOTHERMAL, np.array([Tr]))
    bcs[FACE_YP] = (BC_OUTFLOW_CHAR, np.zeros(0))
    return Problem(name=f"bl{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, lx=lx, lz=lz,
                   y=y, y_eta=ye, y_etaeta=yee, gamma=g, Pr=Pr, R_gas=R, mu_ref=mu_ref,
                   T_ref=1.0, S_suth=S, viscous=True, sensor_mode=SENSOR_HYBRID,
                   theta_star=theta_star, sensor_eps=1.0, forcing=False, bcs=bcs, w0=w0,
                   cfl=0.8, nsteps=nsteps)


def small_boundary_layer(nx: int = 48, ny: int = 32, nz: int = 16, **kw) -> Problem:
    """Parity-sized boundary layer (same recipe, shorter box)."""
    kw.setdefault("lx", 4.0)
    kw.setdefault("ly", 3.0)
    kw.setdefault("lz", 1.5)
    kw.setdefault("beta", 2.0)
    kw.setdefault("re_tau", 120.0)
    return boundary_layer(nx, ny, nz, **kw)


# ----------------------------------------------- decaying isotropic turbulence
def decaying_turbulence(n: int, mach: float, re: float, seed: int,
                        k0: float = 4.0, sensor_mode: int = SENSOR_HYBRID,
                        nsteps: int = 200) -> Problem:
    """Periodic box [0, 2pi)^3 with a seeded solenoidal velocity field.

    Energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2), u_rms = 1 (per component
    rms of 1/sqrt(3) times sqrt(3)), uniform density and pressure,
    Mach = u_rms / c, Re = 1/mu_ref."""
    g = 1.4
    R = 1.0 / (g * mach * mach)
    L = 2.0 * math.pi
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    kk[0, 0, 0] = 1.0
    amp = np.sqrt(kk ** 4 * np.exp(-2.0 * (kk / k0) ** 2)) / kk
    amp[0, 0, 0] = 0.0
    comps = []
    for _ in range(3):
        ph = rng.uniform(0, 2 * math.pi, size=kk.shape)
        comps.append(amp * np.exp(1j * ph))
    # solenoidal projection
    dot = (KX * comps[0] + KY * comps[1] + KZ * comps[2]) / (kk ** 2)
    comps[0] = comps[0] - KX * dot
    comps[1] = comps[1] - KY * dot
    comps[2] = comps[2] - KZ * dot
    vel = [np.real(np.fft.ifftn(c)) for c in comps]
    # divergence-free after taking the real part as well (projection is linear)
    urms = math.sqrt(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    vel = [vv / urms for vv in vel]
    rho = np.ones((n, n, n))
    p = np.full((n, n, n), R)
    w0 = conserved_from_primitive(rho, vel[0], vel[1], vel[2], p, g)
    y, ye, yee = uniform_periodic_y(n, L)
    return Problem(name=f"dit{n}", nx=n, ny=n, nz=n, lx=L, lz=L, y=y, y_eta=ye,
                   y_etaeta=yee, gamma=g, Pr=0.72, R_gas=R, mu_ref=1.0 / re, T_ref=1.0,
                   S_suth=sutherland_S(300.0), viscous=True, sensor_mode=sensor_mode,
                   theta_star=0.1, sensor_eps=1.0, forcing=False, bcs=_periodic_bcs(),
                   w0=w0, cfl=0.8, nsteps=nsteps)


# ----------------------------------------------------------- test problems
def isentropic_vortex_fields(X, Y, t: float = 0.0, strength: float = 5.0,
                             gamma: float = 1.4, center=(5.0, 5.0), period=(10.0, 10.0),
                             uinf=(1.0, 1.0)):
    """Primitive fields of the translating isentropic vortex (R = 1, rho_inf = p_inf = 1).

    The vortex centre moves with the free stream; images in the periodic box
    are summed over the nearest copies so the field is smooth and periodic."""
    rho = np.zeros_like(X)
    cx = (center[0] + uinf[0] * t) % period[0]
    cy = (center[1] + uinf[1] * t) % period[1]
    du = np.zeros_like(X)
    dv = np.zeros_like(X)
    dT = np.zeros_like(X)
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            xb = X - (cx + sx * period[0])
            yb = Y - (cy + sy * period[1])
            r2 = xb * xb + yb * yb
            e = np.exp(0.5 * (1.0 - r2))
            du += -strength / (2 * math.pi) * e * yb
            dv += strength / (2 * math.pi) * e * xb
            dT += -(gamma - 1.0) * strength ** 2 / (8 * gamma * math.pi ** 2) * e * e
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return rho, uinf[0] + du, uinf[1] + dv, p


def isentropic_vortex(n: int, plane: str = "xy", t: float = 0.0, nthin: int = 4,
                      L: float = 10.0) -> Problem:
    """Inviscid periodic problem: the vortex in the given coordinate plane, uniform along the third."""
    g = 1.4
    d = L / n
    c = (np.arange(n) + 0.5) * d
    if plane == "xy":
        nx, ny, nz = n, n, nthin
    elif plane == "xz":
        nx, ny, nz = n, nthin, n
    else:
        nx, ny, nz = nthin, n, n
    lx = L if plane in ("xy", "xz") else nthin * d
    ly = L if plane in ("xy", "yz") else nthin * d
    lz = L if plane in ("xz", "yz") else nthin * d
    shape = (nz, ny, nx)
    A, B = np.meshgrid(c, c, indexing="ij")  # A = first-axis coordinate (slow), B = fast
    # rho,u,v,p in the (a, b) plane where a,b are the plane's two axes in order
    rho2, ua, ub, p2 = isentropic_vortex_fields(B, A, t=t, gamma=g)  # X=B (first axis), Y=A
    # map (first axis, second axis) of the plane to (x,y,z)
    rho = np.zeros(shape); u = np.zeros(shape); v = np.zeros(shape)
    w = np.zeros(shape); p = np.zeros(shape)
    if plane == "xy":
        rho[:] = rho2[None]; p[:] = p2[None]; u[:] = ua[None]; v[:] = ub[None]
    elif plane == "xz":
        rho[:] = rho2[:, None, :]; p[:] = p2[:, None, :]
        u[:] = ua[:, None, :]; w[:] = ub[:, None, :]
    else:
        rho[:] = rho2[:, :, None]; p[:] = p2[:, :, None]
        v[:] = ua[:, :, None]; w[:] = ub[:, :, None]
    w0 = conserved_from_primitive(rho, u, v, w, p, g)
    y, ye, yee = uniform_periodic_y(ny, ly)
    return Problem(name=f"vortex{plane}{n}", nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y=y,
                   y_eta=ye, y_etaeta=yee, gamma=g, Pr=0.72, R_gas=1.0, mu_ref=0.0,
                   viscous=False, sensor_mode=SENSOR_OFF, forcing=False,
                   bcs=_periodic_bcs(), w0=w0, cfl=0.5)


SOD_LEFT = (1.0, 0.0, 1.0)
SOD_RIGHT = (0.125, 0.0, 0.1)


def sod_tube(n: int, axis: int = 0, nthin: int = 4, sensor_mode: int = SENSOR_WENO_ALL,
             theta_star: float = 0.1) -> Problem:
    """Periodic Sod tube of length 2 along `axis`: left state on [0,1), right on [1,2).

    Cell-centred positions s_i = (i + 1/2) * 2/n; the second discontinuity at
    s = 0 == 2 is the mirror image of the first."""
    g = 1.4
    L = 2.0
    d = L / n
    s = (np.arange(n) + 0.5) * d
    left = s < 1.0
    rho1 = np.where(left, SOD_LEFT[0], SOD_RIGHT[0])
    p1 = np.where(left, SOD_LEFT[2], SOD_RIGHT[2])
    dims = [nthin, nthin, nthin]  # (nx, ny, nz)
    dims[axis] = n
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    sl = [None, None, None]
    sl[2 - axis] = slice(None)
    rho = np.broadcast_to(rho1[tuple(sl)], shape).copy()
    p = np.broadcast_to(p1[tuple(sl)], shape).copy()
    z0 = np.zeros(shape)
    w0 = conserved_from_primitive(rho, z0, z0, z0, p, g)
    lens = [nthin * d] * 3
    lens[axis] = L
    y, ye, yee = uniform_periodic_y(ny, lens[1])
    return Problem(name=f"sod{n}_{'xyz'[axis]}", nx=nx, ny=ny, nz=nz, lx=lens[0],
                   lz=lens[2], y=y, y_eta=ye, y_etaeta=yee, gamma=g, R_gas=1.0,
                   mu_ref=0.0, viscous=False, sensor_mode=sensor_mode,
                   theta_star=theta_star, sensor_eps=1.0, forcing=False,
                   bcs=_periodic_bcs(), w0=w0, cfl=0.5)


def random_state(nx: int, ny: int, nz: int, seed: int, amp: float = 0.2,
                 mach: float = 0.8) -> np.ndarray:
    """A smooth-ish random positive state (used by brute-force and parity tests)."""
    g = 1.4
    R = 1.0 / (g * mach * mach)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    rho = 1.0 + amp * rng.uniform(-1, 1, shape)
    u = amp * 3 * rng.uniform(-1, 1, shape)
    v = amp * 3 * rng.uniform(-1, 1, shape)
    w = amp * 3 * rng.uniform(-1, 1, shape)
    T = 1.0 + amp * rng.uniform(-1, 1, shape)
    p = rho * R * T
    return conserved_from_primitive(rho, u, v, w, p, g)


def with_state(pr: Problem, w0: np.ndarray, **changes) -> Problem:
    """A copy of `pr` with a new initial state and optional field overrides."""
    return dataclasses.replace(pr, w0=np.ascontiguousarray(w0, dtype=np.float64), **changes)


def small_channel(nx=24, ny=20, nz=12, **kw) -> Problem:
    """The channel configuration at a size the oracle finishes in seconds."""
    return channel(nx, ny, nz, **kw)


def small_sbli(nx=64, ny=32, nz=8, **kw) -> Problem:
    """The shock/boundary-layer box at a size the oracle finishes in seconds."""
    return sbli(nx, ny, nz, **kw)


# ------------------------------------------------------------ serving requests
def convected_turbulence(n: int, mach: float, re: float, seed: int, turb_mach: float = 0.3,
                         sensor_mode: int = SENSOR_HYBRID, nsteps: int = 200) -> Problem:
    """Periodic decaying turbulence carried by a uniform stream.

    The stream has unit velocity along x and Mach number `mach` (sound
    speed 1/mach at T = 1); the solenoidal fluctuation field of
    `decaying_turbulence` is scaled to u_rms = turb_mach times the sound
    speed; density and pressure are uniform; Re = 1/mu_ref."""
    base = decaying_turbulence(n, mach=1.0, re=re, seed=seed, sensor_mode=sensor_mode,
                               nsteps=nsteps)
    g = 1.4
    R = 1.0 / (g * mach * mach)
    c0 = 1.0 / mach
    rho = base.w0[0]
    u, v, w = (base.w0[1] / rho, base.w0[2] / rho, base.w0[3] / rho)
    s = turb_mach * c0
    w0 = conserved_from_primitive(rho, 1.0 + s * u, s * v, s * w, np.full_like(rho, R), g)
    return dataclasses.replace(base, name=f"cturb{n}", R_gas=R, mu_ref=1.0 / re, w0=w0)


@dataclasses.dataclass
class RequestSpec:
    rid: int
    arrival: float      # seconds after the start of the trace
    kind: str           # "turbulence" or "channel"
    n: int              # cubic grid n^3
    mach: float
    re: float
    seed: int
    nsteps: int = 200


def serving_trace(n_requests: int = 64, rate: float = 4.0, nmin: int = 32, nmax: int = 192,
                  mach_range=(0.1, 3.0), re_range=(500.0, 5000.0), nsteps: int = 200,
                  seed_index: int = 4, burst: bool = False) -> List[RequestSpec]:
    """Poisson arrivals (exponential gaps of mean 1/rate; all at t = 0 when
    burst), kind uniform over {turbulence, channel}, n uniform in
    [nmin, nmax] (even), Mach and Re uniform in their ranges."""
    rng = _rng(seed_index)
    t = 0.0
    out = []
    for r in range(n_requests):
        if not burst:
            t += float(rng.exponential(1.0 / rate))
        kind = "turbulence" if rng.uniform() < 0.5 else "channel"
        n = int(rng.integers(nmin // 2, nmax // 2 + 1)) * 2
        mach = float(rng.uniform(*mach_range))
        re = float(rng.uniform(*re_range))
        out.append(RequestSpec(r, 0.0 if burst else t, kind, n, mach, re,
                               BASE_SEED + 100 + r, nsteps))
    return out


def request_problem(spec: RequestSpec) -> Problem:
    """Initial field and parameters of one serving request."""
    if spec.kind == "turbulence":
        return convected_turbulence(spec.n, spec.mach, spec.re, spec.seed, nsteps=spec.nsteps)
    pr = channel(spec.n, spec.n, spec.n, mach_b=spec.mach, re_b=spec.re,
                 seed_index=spec.seed - BASE_SEED, nsteps=spec.nsteps)
    return dataclasses.replace(pr, name=f"chan{spec.n}")
