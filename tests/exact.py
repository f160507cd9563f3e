"""Exact and analytic solutions used to pin the oracle (test utilities).

* exact solution of the Riemann problem for the Euler equations of a
  perfect gas (the textbook pressure-function method: Newton iteration on
  the star-region pressure, then sampling of the self-similar solution);
* manufactured smooth periodic fields with the exact continuous right-hand
  side of the compressible Navier-Stokes equations (Sec. 2 of the paper),
  obtained symbolically with sympy in *divergence* form, so that they pin
  the Laplacian-form expansion used by the discretisation.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


# ------------------------------------------------------------------ Riemann
def _pfun(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _pfun(p, rl, pl, cl, g)
        fr, dfr = _pfun(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-10)
        if abs(pn - p) / (0.5 * (pn + p)) < 1e-14:
            p = pn
            break
        p = pn
    fl, _ = _pfun(p, rl, pl, cl, g)
    fr, _ = _pfun(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, s, g=1.4):
    """Exact (rho, u, p) at similarity coordinates s = x/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = riemann_star(left, right, g)
    out = np.zeros((3,) + np.shape(s))
    gm = (g - 1.0) / (g + 1.0)
    for idx, si in np.ndenumerate(s):
        if si <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if si <= sl:
                    val = (rl, ul, pl)
                else:
                    val = (rl * (ps / pl + gm) / (gm * ps / pl + 1), us, ps)
            else:  # left rarefaction
                shl = ul - cl
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - csl
                if si <= shl:
                    val = (rl, ul, pl)
                elif si >= stl:
                    val = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - si))
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + si)
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    val = (rho, uu, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if si >= sr:
                    val = (rr, ur, pr)
                else:
                    val = (rr * (ps / pr + gm) / (gm * ps / pr + 1), us, ps)
            else:
                shr = ur + cr
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + csr
                if si >= shr:
                    val = (rr, ur, pr)
                elif si <= str_:
                    val = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - si))
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + si)
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    val = (rho, uu, pr * (c / cr) ** (2 * g / (g - 1)))
        out[(slice(None),) + idx] = val
    return out


# -------------------------------------------------------- manufactured fields
@lru_cache(maxsize=4)
def manufactured_rhs(gamma: float, R_gas: float, Pr: float, mu_ref: float, S: float):
    """Return numpy callables (prim(x,y,z) -> rho,u,v,w,p ; euler(x,y,z) -> 5 fields ;
    viscous(x,y,z) -> 5 fields) of the exact continuous right-hand side split
    into inviscid and viscous parts, for a fixed smooth 2pi-periodic field."""
    import sympy as sp

    x, y, z = sp.symbols("x y z", real=True)
    rho = 1 + sp.Rational(1, 5) * sp.sin(x) * sp.cos(y) + sp.Rational(1, 10) * sp.cos(z)
    u = sp.Rational(1, 2) * sp.sin(y) + sp.Rational(3, 10) * sp.cos(x + z)
    v = sp.Rational(2, 5) * sp.cos(x) * sp.sin(z) + sp.Rational(1, 5) * sp.sin(y)
    w = sp.Rational(3, 10) * sp.sin(x + y) + sp.Rational(1, 5) * sp.cos(z)
    T = 1 + sp.Rational(1, 5) * sp.cos(x) * sp.sin(y + z)
    g = sp.Float(gamma, 30)
    R = sp.Float(R_gas, 30)
    p = rho * R * T
    cv = R / (g - 1)
    cp = g * R / (g - 1)
    E = cv * T + (u ** 2 + v ** 2 + w ** 2) / 2
    vel = [u, v, w]
    X = [x, y, z]
    # inviscid
    e_mass = -sum(sp.diff(rho * vel[j], X[j]) for j in range(3))
    e_mom = [-sum(sp.diff(rho * vel[i] * vel[j] + (p if i == j else 0), X[j]) for j in range(3))
             for i in range(3)]
    e_en = -sum(sp.diff(vel[j] * (rho * E + p), X[j]) for j in range(3))
    # viscous, divergence form
    t = T  # T_ref = 1
    mu = sp.Float(mu_ref, 30) * t * sp.sqrt(t) * (1 + sp.Float(S, 30)) / (t + sp.Float(S, 30))
    kcond = cp * mu / sp.Float(Pr, 30)
    div = sum(sp.diff(vel[k], X[k]) for k in range(3))
    sig = [[mu * (sp.diff(vel[i], X[j]) + sp.diff(vel[j], X[i])
                  - (sp.Rational(2, 3) * div if i == j else 0)) for j in range(3)] for i in range(3)]
    v_mom = [sum(sp.diff(sig[i][j], X[j]) for j in range(3)) for i in range(3)]
    v_en = sum(sp.diff(sum(sig[i][j] * vel[i] for i in range(3)), X[j]) for j in range(3)) \
        + sum(sp.diff(kcond * sp.diff(T, X[j]), X[j]) for j in range(3))
    mods = ["numpy"]
    prim = sp.lambdify((x, y, z), [rho, u, v, w, p], mods)
    euler = sp.lambdify((x, y, z), [e_mass] + e_mom + [e_en], mods)
    visc = sp.lambdify((x, y, z), [sp.Integer(0)] + v_mom + [v_en], mods)
    return prim, euler, visc


def eval_fields(fn, X, Y, Z):
    out = fn(X, Y, Z)
    return np.stack([np.broadcast_to(np.asarray(o, dtype=np.float64), X.shape) for o in out])
