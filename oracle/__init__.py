"""FP64 CPU oracle for the compressible Navier-Stokes right-hand side and RK3 step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product library never does.  It is an
independent implementation (plain C in cdns_oracle.c, padded ghost arrays,
literal formulas of the paper) and shares no code with the GPU path.  Both
sides receive the same seeded inputs from the `problems` package.

Parity status: every operator is pinned by CPU tests against closed forms,
invariants or exact solutions (see tests/test_oracle_*.py).  The
characteristic Lax-Friedrichs WENO flux is pinned by its reduction to the
scalar reconstruction for an entropy wave, exact stationary contacts,
design-order convergence with WENO at every interface, splitting constants
against independently computed Jacobian eigenvalues and its exact stencil
(tests/test_oracle_pins_flux.py); the wall and imposed-shock ghost nodes by
their closed forms and by the equivalent mirrored periodic domain; the
volume totals by plain sums.  The characteristic outflow boundary is pinned
only by a behaviour check (acoustic pulse reflection), so it is "parity
unpinned" against the paper; the digital-filter inflow generator is pinned
by the published SplitMix64 reference outputs and by its statistics (unit
variance of the filtered field, prescribed Reynolds stresses, filter and
time correlations), its constants are readings (the paper gives the method
only).  The scheme-order variants (central order 2L for L = 1, 2, 3; WENO
order 2r - 1 for r = 2, 3, 4) are pinned in tests/test_oracle_orders.py by
Taylor-derived weights, polynomial definitions of the WENO candidates and
indicators, design-order convergence, conservation and kinetic-energy
identities and the exact Sod solution.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdns_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

T_CONV, T_PRES, T_VISC, T_FORCE, T_ALL = 1, 2, 4, 8, 15

ORA_OK, ORA_EINVAL, ORA_ENOMEM, ORA_ESTATE, ORA_EUNSUP = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("lz", ctypes.c_double),
        ("y_eta", ctypes.POINTER(ctypes.c_double)),
        ("y_etaeta", ctypes.POINTER(ctypes.c_double)),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("R_gas", ctypes.c_double),
        ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("S_suth", ctypes.c_double),
        ("viscous", ctypes.c_int32), ("sensor_mode", ctypes.c_int32),
        ("theta_star", ctypes.c_double), ("sensor_eps", ctypes.c_double),
        ("forcing", ctypes.c_int32), ("terms", ctypes.c_int32),
        ("bc_kind", ctypes.c_int32 * 6),
        ("bc_params", ctypes.POINTER(ctypes.c_double) * 6),
        ("bc_nparams", ctypes.c_int32 * 6),
        ("df_plane", ctypes.POINTER(ctypes.c_double)),
        ("central_L", ctypes.c_int32), ("weno_r", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(_Problem)
        lib.ora_rhs.argtypes = [pp, dp, dp, dp, u8p, u8p, dp]
        lib.ora_rhs.restype = ctypes.c_int
        lib.ora_dt.argtypes = [pp, dp, ctypes.c_double, dp]
        lib.ora_dt.restype = ctypes.c_int
        lib.ora_advance.argtypes = [pp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.ora_advance.restype = ctypes.c_int
        lib.ora_rk_stage.argtypes = [ctypes.c_size_t, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        lib.ora_rk_stage.restype = None
        lib.ora_weno5.argtypes = [dp]
        lib.ora_weno5.restype = ctypes.c_double
        lib.ora_weno.argtypes = [ctypes.c_int, dp]
        lib.ora_weno.restype = ctypes.c_double
        lib.ora_weno_parts.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.ora_weno_parts.restype = None
        lib.ora_eigenvectors.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.ora_eigenvectors.restype = None
        lib.ora_totals.argtypes = [pp, dp, dp]
        lib.ora_totals.restype = ctypes.c_int
        lib.ora_extrema.argtypes = [pp, dp, dp]
        lib.ora_extrema.restype = ctypes.c_int
        lib.ora_iface_flux.argtypes = [pp, dp, ctypes.c_int, dp]
        lib.ora_iface_flux.restype = ctypes.c_int
        lib.ora_num_threads.argtypes = []
        lib.ora_num_threads.restype = ctypes.c_int
        lib.ora_set_threads.argtypes = [ctypes.c_int]
        lib.ora_set_threads.restype = ctypes.c_int
        lib.ora_stats.argtypes = [pp, dp, dp]
        lib.ora_stats.restype = ctypes.c_int
        lib.ora_stats_means.argtypes = [pp, dp, ctypes.c_long, ctypes.c_int, dp]
        lib.ora_stats_means.restype = ctypes.c_int
        lib.ora_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.ora_splitmix64.restype = ctypes.c_uint64
        lib.ora_df_update.argtypes = [pp, ctypes.c_uint64, ctypes.c_double, ctypes.c_int, dp, dp,
                                      dp]
        lib.ora_df_update.restype = ctypes.c_int
        lib.ora_df_coeffs.argtypes = [pp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      dp, dp, dp]
        lib.ora_df_coeffs.restype = ctypes.c_int
        lib.ora_ghosts_y.argtypes = [pp, dp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int)]
        lib.ora_ghosts_y.restype = ctypes.c_int
        lib.ora_lf_alpha.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, dp]
        lib.ora_lf_alpha.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Marshalled:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, pr, terms: int = T_ALL):
        self.keep = []
        s = _Problem()
        s.nx, s.ny, s.nz = pr.nx, pr.ny, pr.nz
        s.lx, s.lz = pr.lx, pr.lz
        ye = np.ascontiguousarray(pr.y_eta, dtype=np.float64)
        yee = np.ascontiguousarray(pr.y_etaeta, dtype=np.float64)
        self.keep += [ye, yee]
        s.y_eta, s.y_etaeta = _dptr(ye), _dptr(yee)
        s.gamma, s.Pr, s.R_gas = pr.gamma, pr.Pr, pr.R_gas
        s.mu_ref, s.T_ref, s.S_suth = pr.mu_ref, pr.T_ref, pr.S_suth
        s.viscous = int(bool(pr.viscous))
        s.sensor_mode = int(pr.sensor_mode)
        s.theta_star, s.sensor_eps = pr.theta_star, pr.sensor_eps
        s.forcing = int(bool(pr.forcing))
        s.terms = int(terms)
        s.central_L, s.weno_r = scheme_params(pr)
        for f, (kind, params) in enumerate(pr.bcs):
            arr = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
            if arr.size == 0:
                arr = np.zeros(1)
                n = 0
            else:
                n = arr.size
            self.keep.append(arr)
            s.bc_kind[f] = int(kind)
            s.bc_params[f] = _dptr(arr)
            s.bc_nparams[f] = n
        self.s = s


def scheme_params(pr):
    """(L, r) of a problem: central order 2L, WENO order 2r - 1 (defaults
    4 and 5 when the problem does not name them)."""
    co = int(getattr(pr, "central_order", 4))
    wo = int(getattr(pr, "weno_order", 5))
    if co not in (2, 4, 6) or wo not in (3, 5, 7):
        raise ValueError(f"unsupported scheme orders central {co}, WENO {wo}")
    return co // 2, (wo + 1) // 2


def _check(st: int, what: str):
    if st != ORA_OK:
        raise OracleError(f"{what} failed with status {st}")


def rhs(pr, w: Optional[np.ndarray] = None, terms: int = T_ALL, want_flags: bool = False):
    """R(w) on the whole grid.  Returns R (5,nz,ny,nx); with want_flags also
    (theta, node_flags, iface_flags, forcing)."""
    lib = _load()
    w = np.ascontiguousarray(pr.w0 if w is None else w, dtype=np.float64)
    shp = (pr.nz, pr.ny, pr.nx)
    r = np.zeros((5,) + shp)
    theta = np.zeros(shp)
    nfl = np.zeros(shp, dtype=np.uint8)
    ifl = np.zeros(shp, dtype=np.uint8)
    f = ctypes.c_double(0.0)
    m = _Marshalled(pr, terms)
    st = lib.ora_rhs(ctypes.byref(m.s), _dptr(w), _dptr(r), _dptr(theta),
                     nfl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                     ifl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(f))
    _check(st, "ora_rhs")
    if want_flags:
        return r, theta, nfl, ifl, f.value
    return r


def dt(pr, w: Optional[np.ndarray] = None, cfl: Optional[float] = None) -> float:
    lib = _load()
    w = np.ascontiguousarray(pr.w0 if w is None else w, dtype=np.float64)
    out = ctypes.c_double(0.0)
    m = _Marshalled(pr)
    _check(lib.ora_dt(ctypes.byref(m.s), _dptr(w), float(pr.cfl if cfl is None else cfl),
                      ctypes.byref(out)), "ora_dt")
    return out.value


def advance(pr, nsteps: int, w: Optional[np.ndarray] = None, cfl: Optional[float] = None,
            dt_fixed: float = 0.0, return_dts: bool = False):
    """Advance a copy of the state by nsteps RK3 steps."""
    lib = _load()
    w = np.array(pr.w0 if w is None else w, dtype=np.float64, copy=True, order="C")
    dts = np.zeros(max(nsteps, 1))
    m = _Marshalled(pr)
    st = lib.ora_advance(ctypes.byref(m.s), _dptr(w), int(nsteps),
                         float(pr.cfl if cfl is None else cfl), float(dt_fixed), _dptr(dts))
    _check(st, "ora_advance")
    if return_dts:
        return w, dts[:nsteps]
    return w


def rk_stage(w: np.ndarray, r: np.ndarray, rprev: np.ndarray, dt_: float, stage: int) -> np.ndarray:
    """One low-storage RK3 stage on flat float64 arrays."""
    lib = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    rprev = np.ascontiguousarray(rprev, dtype=np.float64)
    out = np.empty_like(w)
    lib.ora_rk_stage(w.size, _dptr(w), _dptr(r), _dptr(rprev), float(dt_), int(stage), _dptr(out))
    return out


def weno5(v) -> float:
    lib = _load()
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    assert a.size == 5
    return lib.ora_weno5(_dptr(a))


def weno(r: int, v) -> float:
    """WENO-JS reconstruction of order 2r-1 at the right face of the middle
    cell of the 2r-1 values v."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    assert a.size == 2 * r - 1
    return lib.ora_weno(int(r), _dptr(a))


def weno_parts(r: int, v):
    """(candidate face values q_k, smoothness indicators beta_k) of the
    reconstruction of order 2r-1."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    assert a.size == 2 * r - 1
    q = np.zeros(4)
    b = np.zeros(4)
    lib.ora_weno_parts(int(r), _dptr(a), _dptr(q), _dptr(b))
    return q[:r], b[:r]


def eigenvectors(gamma: float, d: int, u: float, v: float, w: float, Ht: float):
    """(R, L) in natural component order: R[component, wave], L[wave, component]."""
    lib = _load()
    R = np.zeros(25)
    L = np.zeros(25)
    lib.ora_eigenvectors(gamma, d, u, v, w, Ht, _dptr(R), _dptr(L))
    return R.reshape(5, 5), L.reshape(5, 5)


def totals(pr, w: np.ndarray) -> np.ndarray:
    """Volume integrals: mass, momentum (3), total energy, kinetic energy."""
    lib = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(6)
    m = _Marshalled(pr)
    _check(lib.ora_totals(ctypes.byref(m.s), _dptr(w), _dptr(out)), "ora_totals")
    return out


def extrema(pr, w: np.ndarray) -> np.ndarray:
    """(min rho, min p, max Mach, number of non-finite conserved values)."""
    lib = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(4)
    m = _Marshalled(pr)
    _check(lib.ora_extrema(ctypes.byref(m.s), _dptr(w), _dptr(out)), "ora_extrema")
    return out


def iface_flux(pr, d: int, w: Optional[np.ndarray] = None) -> np.ndarray:
    """Interface fluxes along direction d as used by the right-hand side
    (interface i+1/2 stored at node i), shape (5, nz, ny, nx)."""
    lib = _load()
    w = np.ascontiguousarray(pr.w0 if w is None else w, dtype=np.float64)
    out = np.zeros((5, pr.nz, pr.ny, pr.nx))
    m = _Marshalled(pr)
    _check(lib.ora_iface_flux(ctypes.byref(m.s), _dptr(w), int(d), _dptr(out)), "ora_iface_flux")
    return out


def ghosts_y(pr, face: int, w: Optional[np.ndarray] = None):
    """Ghost layers of y face `face` (2: y-, 3: y+) as filled for the
    right-hand side: array (5, hw, nz, nx + 2 hw), layer s-1 = ghost s,
    x index offset by hw."""
    lib = _load()
    w = np.ascontiguousarray(pr.w0 if w is None else w, dtype=np.float64)
    hw_max = 4
    buf = np.zeros(5 * hw_max * pr.nz * (pr.nx + 2 * hw_max))
    hw = ctypes.c_int(0)
    m = _Marshalled(pr)
    st = lib.ora_ghosts_y(ctypes.byref(m.s), _dptr(w), int(face), _dptr(buf), ctypes.byref(hw))
    if st not in (ORA_OK, ORA_ESTATE):
        _check(st, "ora_ghosts_y")
    h = hw.value
    return buf[:5 * h * pr.nz * (pr.nx + 2 * h)].reshape(5, h, pr.nz, pr.nx + 2 * h)


def lf_alpha(pr, d: int, i: int, j: int, k: int, w: Optional[np.ndarray] = None) -> np.ndarray:
    """Lax-Friedrichs splitting constants (waves u-c, u, u, u, u+c) of the
    shock-capturing flux at interface i+1/2 of direction d."""
    lib = _load()
    w = np.ascontiguousarray(pr.w0 if w is None else w, dtype=np.float64)
    out = np.zeros(5)
    m = _Marshalled(pr)
    _check(lib.ora_lf_alpha(ctypes.byref(m.s), _dptr(w), int(d), int(i), int(j), int(k),
                            _dptr(out)), "ora_lf_alpha")
    return out


def num_threads() -> int:
    return _load().ora_num_threads()


def set_threads(n: int) -> int:
    """Thread count of the oracle's parallel loops from now on (timing only:
    results do not depend on it); returns the previous count."""
    return int(_load().ora_set_threads(int(n)))


def splitmix64(seed: int, n: int) -> int:
    """Output n (n >= 1) of the SplitMix64 generator seeded with `seed`."""
    return int(_load().ora_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(n)))


def df_update(pr, key: int, dt: float, first: bool, psi: Optional[np.ndarray] = None):
    """One update of the digital-filter inflow generator of `pr` (face x-).
    Returns (psi [3][nz][ny], conserved plane [5][nz][ny], velocity
    fluctuations [3][nz][ny])."""
    lib = _load()
    psi = np.zeros((3, pr.nz, pr.ny)) if psi is None else np.ascontiguousarray(psi, np.float64).copy()
    plane = np.zeros((5, pr.nz, pr.ny))
    fl = np.zeros((3, pr.nz, pr.ny))
    m = _Marshalled(pr)
    _check(lib.ora_df_update(ctypes.byref(m.s), ctypes.c_uint64(key), float(dt), int(bool(first)),
                             _dptr(psi), _dptr(plane), _dptr(fl)), "ora_df_update")
    return psi, plane, fl


def df_coeffs(pr):
    """Derived coefficients of the digital-filter inflow of `pr` (face x-):
    (b_y, b_z, lower triangular factor [6][ny] as a11, a21, a22, a31, a32,
    a33)."""
    lib = _load()
    by = np.zeros(2 * pr.ny + 3)
    bz = np.zeros(2 * pr.nz + 3)
    chol = np.zeros((6, pr.ny))
    ny_, nz_ = ctypes.c_int(0), ctypes.c_int(0)
    m = _Marshalled(pr)
    _check(lib.ora_df_coeffs(ctypes.byref(m.s), ctypes.byref(ny_), ctypes.byref(nz_), _dptr(by),
                             _dptr(bz), _dptr(chol)), "ora_df_coeffs")
    return by[:2 * ny_.value + 1], bz[:2 * nz_.value + 1], chol


STAT_NAMES = ["rho", "rho_u", "rho_v", "rho_w", "rho_uu", "rho_vv", "rho_ww", "rho_uv", "u", "uu",
              "T", "rho_T", "TT", "p", "pp", "rho_rho"]


def stats(pr, w: np.ndarray, acc: Optional[np.ndarray] = None) -> np.ndarray:
    """Spanwise sums of the statistics products of state w added to acc
    (shape (16, ny, nx)); returns acc."""
    lib = _load()
    acc = np.zeros((16, pr.ny, pr.nx)) if acc is None else acc
    w = np.ascontiguousarray(w, dtype=np.float64)
    m = _Marshalled(pr)
    _check(lib.ora_stats(ctypes.byref(m.s), _dptr(w), _dptr(acc)), "ora_stats")
    return acc


MEAN_NAMES = ["rho", "u_favre", "v_favre", "w_favre", "R11", "R22", "R33", "R12", "u", "u_rms",
              "T", "T_favre", "T_rms", "p", "p_rms", "rho_rms"]


def stats_means(pr, acc: np.ndarray, samples: int, average_x: bool = False) -> dict:
    """Mean fields (MEAN_NAMES) from sums accumulated by `stats` over
    `samples` states: arrays over (y, x), or over y with average_x."""
    lib = _load()
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    shp = (16, pr.ny) if average_x else (16, pr.ny, pr.nx)
    out = np.zeros(shp)
    m = _Marshalled(pr)
    _check(lib.ora_stats_means(ctypes.byref(m.s), _dptr(acc), int(samples), int(bool(average_x)),
                               _dptr(out)), "ora_stats_means")
    return {name: out[q] for q, name in enumerate(MEAN_NAMES)}
