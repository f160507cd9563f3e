"""Pins of the oracle's boundary-layer machinery (Sec. 3.2): the
counter-based generator, the digital-filter inflow statistics, the
characteristic outflow on y faces, and the mean-profile recipe.

The statistics are checked against what the construction fixes exactly
in expectation: unit variance of the filtered field (coefficients with unit
sum of squares), its spatial correlation (sum_l b_l b_{l+r} for filtered
white noise), the time correlation E = exp(-pi dt/(2T)) with stationary
variance, and the prescribed Reynolds stresses through the Cholesky
factor; tolerances cover the sampling error of the sample sizes used.
"""
import math
import os

import numpy as np
import pytest

import oracle
import problems as P


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_splitmix64_published_outputs():
    """Reference outputs of the published SplitMix64 generator
    (tests/golden/splitmix64_reference.txt, with its citation)."""
    rows = [line.split() for line in open(os.path.join(GOLDEN, "splitmix64_reference.txt"))
            if line.strip() and not line.startswith("#")]
    assert len(rows) >= 4
    for seed, n, out in rows:
        assert oracle.splitmix64(int(seed), int(n)) == int(out), (seed, n)


def _plane_problem(ny=48, nz=64, ny_len=3.0, nz_len=4.0, t_lag=0.5, stresses=None):
    """A channel-shaped problem whose x- face carries a digital-filter
    inflow with uniform mean state and the given constant stresses."""
    pr = P.small_channel(16, ny, nz)
    mean = np.stack([np.ones(ny), np.full(ny, 1.0), np.zeros(ny), np.zeros(ny),
                     np.full(ny, pr.R_gas)])
    R11, R22, R33, R12 = stresses if stresses is not None else (4.0, 2.0, 1.0, -1.0)
    rs = np.stack([np.full(ny, R11), np.full(ny, R22), np.full(ny, R33), np.full(ny, R12),
                   np.zeros(ny), np.zeros(ny)])
    params = P.df_inflow_params(mean, rs, ny_len, nz_len, t_lag, 777)
    bcs = list(pr.bcs)
    bcs[P.FACE_XM] = (P.BC_DF_INFLOW, params)
    bcs[P.FACE_XP] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    import dataclasses
    pr = dataclasses.replace(pr, bcs=bcs)
    by, bz, _ = oracle.df_coeffs(pr)
    return pr, by, bz


@pytest.mark.parametrize("n", [1.0, 2.5, 4.0, 7.3])
def test_df_filter_coefficients_give_the_integral_length(n):
    """The filtered white noise has the autocorrelation rho(r) = sum_l b_l
    b_(l+r); with the Gaussian coefficients its integral length
    int_0^inf rho(r) dr (trapezoidal over the lags) is the prescribed n grid
    spacings (Klein, Sadiki and Janicka 2003, the digital filter's design
    rule) and rho(0) = 1 (unit variance); the half-width is ceil(2 n)."""
    pr, by, bz = _plane_problem(ny=48, nz=64, ny_len=n, nz_len=n)
    for b in (by, bz):
        half = (len(b) - 1) // 2
        assert half == max(1, math.ceil(2 * n))
        assert np.allclose(b, b[::-1], rtol=0, atol=0)               # symmetric
        rho = np.array([np.sum(b[: len(b) - r] * b[r:]) for r in range(len(b))])
        assert abs(rho[0] - 1.0) <= 1e-14
        length = rho.sum() - 0.5 * rho[0]
        # the truncation at 2n drops the tail beyond exp(-4 pi) of the kernel
        assert abs(length - n) <= (1e-3 * n if n >= 2 else 0.08), (n, length)


def test_df_stress_factor_reproduces_the_stresses():
    """Lund's factor a of the Reynolds stresses satisfies a a^T = R for
    positive definite tensors, and zeroes the rows of a vanishing stress
    (the free stream outside the layer)."""
    rng = np.random.Generator(np.random.PCG64(5))
    ny = 48
    rs = np.zeros((6, ny))
    for j in range(ny - 4):
        m = rng.normal(size=(3, 3))
        R = m @ m.T + 0.1 * np.eye(3)
        rs[:, j] = [R[0, 0], R[1, 1], R[2, 2], R[0, 1], R[0, 2], R[1, 2]]
    pr0 = P.small_channel(16, ny, 32)
    mean = np.stack([np.ones(ny), np.ones(ny), np.zeros(ny), np.zeros(ny), np.full(ny, pr0.R_gas)])
    params = P.df_inflow_params(mean, rs, 2.0, 2.0, 0.5, 1)
    bcs = list(pr0.bcs)
    bcs[P.FACE_XM] = (P.BC_DF_INFLOW, params)
    bcs[P.FACE_XP] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    import dataclasses
    pr = dataclasses.replace(pr0, bcs=bcs)
    _, _, a = oracle.df_coeffs(pr)
    for j in range(ny):
        A = np.array([[a[0, j], 0, 0], [a[1, j], a[2, j], 0], [a[3, j], a[4, j], a[5, j]]])
        R = np.array([[rs[0, j], rs[3, j], rs[4, j]], [rs[3, j], rs[1, j], rs[5, j]],
                      [rs[4, j], rs[5, j], rs[2, j]]])
        assert np.abs(A @ A.T - R).max() <= 1e-13 * max(1.0, np.abs(R).max())
    assert np.all(a[:, ny - 4:] == 0.0)


def test_df_filtered_field_variance_and_spatial_correlation():
    pr, by, bz = _plane_problem()
    samples = []
    for key in range(8):
        psi, _, _ = oracle.df_update(pr, key, 0.0, True)
        samples.append(psi)
    s = np.stack(samples)  # [key][c][k][j]
    assert abs(s.mean()) < 0.05
    assert abs(s.var() - 1.0) < 0.06
    # correlation at lag r along y (j) and z (k): filtered white noise
    for r in (1, 2, 4):
        expect_y = float(np.sum(by[:-r] * by[r:]))
        got_y = float(np.mean(s[..., :-r] * s[..., r:]))
        assert abs(got_y - expect_y) < 0.06, (r, got_y, expect_y)
        expect_z = float(np.sum(bz[:-r] * bz[r:]))
        got_z = float(np.mean(s[:, :, :-r, :] * s[:, :, r:, :]))
        assert abs(got_z - expect_z) < 0.06, (r, got_z, expect_z)


def test_df_time_correlation_and_stationary_variance():
    pr, _, _ = _plane_problem(ny=32, nz=32, t_lag=0.5)
    dt = 0.1
    E = math.exp(-math.pi * dt / (2 * 0.5))
    psi, _, _ = oracle.df_update(pr, 0, 0.0, True)
    seq = [psi]
    for key in range(1, 40):
        psi, _, _ = oracle.df_update(pr, key, dt, False, psi)
        seq.append(psi)
    s = np.stack(seq)
    assert abs(s.var() - 1.0) < 0.08
    lag1 = float(np.mean(s[1:] * s[:-1]))
    assert abs(lag1 - E) < 0.06, (lag1, E)


def test_df_velocity_fluctuations_have_the_prescribed_stresses():
    R11, R22, R33, R12 = 4.0, 2.0, 1.0, -1.0
    pr, _, _ = _plane_problem(stresses=(R11, R22, R33, R12))
    fl = np.stack([oracle.df_update(pr, key, 0.0, True)[2] for key in range(8)])
    du, dv, dw = fl[:, 0], fl[:, 1], fl[:, 2]
    assert abs(np.mean(du * du) / R11 - 1) < 0.07
    assert abs(np.mean(dv * dv) / R22 - 1) < 0.07
    assert abs(np.mean(dw * dw) / R33 - 1) < 0.07
    assert abs(np.mean(du * dv) - R12) < 0.15
    assert abs(np.mean(du * dw)) < 0.15 and abs(np.mean(dv * dw)) < 0.15


def test_df_plane_obeys_the_strong_reynolds_analogy():
    pr, _, _ = _plane_problem()
    _, plane, fl = oracle.df_update(pr, 3, 0.0, True)
    rho, mu, mv, mw, E = plane
    u = mu / rho
    cv = pr.R_gas / (pr.gamma - 1)
    T = (E / rho - 0.5 * (u ** 2 + (mv / rho) ** 2 + (mw / rho) ** 2)) / cv
    p = rho * pr.R_gas * T
    cp = pr.gamma * cv
    np.testing.assert_allclose(p, pr.R_gas, rtol=1e-12)           # constant pressure
    np.testing.assert_allclose(u - 1.0, fl[0], atol=1e-12)         # u = u_mean + u'
    np.testing.assert_allclose(cp * (T - 1.0) + 1.0 * fl[0], 0.0, atol=1e-12)  # c_p T' = -u u'


def test_uniform_flow_leaves_through_top_outflow_unchanged():
    # uniform stream with an upward component: the top characteristic
    # outflow must not disturb it (all gradients vanish)
    pr = P.small_boundary_layer(24, 16, 8)
    import dataclasses
    shape = (pr.nz, pr.ny, pr.nx)
    w0 = P.conserved_from_primitive(np.ones(shape), np.full(shape, 0.5), np.full(shape, 0.3),
                                    np.zeros(shape), np.full(shape, pr.R_gas), pr.gamma)
    bcs = list(pr.bcs)
    bcs[P.FACE_XM] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    bcs[P.FACE_YM] = (P.BC_OUTFLOW_CHAR, np.zeros(0))
    prb = dataclasses.replace(pr, bcs=bcs, w0=w0, viscous=False, sensor_mode=P.SENSOR_OFF)
    r = oracle.rhs(prb)
    r = r[0] if isinstance(r, tuple) else r
    assert np.abs(r).max() < 1e-12


def test_mean_profile_recipe():
    pr = P.boundary_layer(32, 96, 8)
    y = pr.y
    rho = pr.w0[0][0, :, 0]
    u = pr.w0[1][0, :, 0] / rho
    # inner law: Musker's profile approaches the log law in the overlap
    yp = np.array([80.0, 150.0])
    np.testing.assert_allclose(P.musker_uplus(yp), np.log(yp) / 0.41 + 5.0, rtol=0.03)
    assert abs(float(P.musker_uplus(0.0))) < 1e-3
    # the van Driest integral of the compressible profile gives back the
    # incompressible one: u_vd = int sqrt(rho/rho_w) du
    inside = y < 1.0
    rho_w = 1.0 / (1.0 + 0.2 * 0.72 ** (1 / 3) * 4.0)
    uu = np.concatenate([[0.0], u[inside]])
    rr = np.concatenate([[rho_w], rho[inside]])
    uvd = np.concatenate([[0.0], np.cumsum(0.5 * (np.sqrt(rr[1:] / rho_w) + np.sqrt(rr[:-1] / rho_w))
                                            * np.diff(uu))])[1:]
    a = math.sqrt((1.0 / rho_w - 1.0) * rho_w)
    np.testing.assert_allclose(uvd, np.arcsin(a * u[inside]) / a, rtol=2e-3, atol=2e-3)
    assert abs(u[inside][-1] - 0.99) < 0.05 and u.max() <= 1.0
