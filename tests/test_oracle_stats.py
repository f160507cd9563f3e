"""Pin of the oracle's running statistics: spanwise sums of a field with a
known z-structure, u = U(y) + A sin(2 pi m z / L_z), uniform density and
pressure.  Over a full period of equally spaced nodes the sum of sin is
zero and the sum of sin^2 is nz/2, so the means and variances are closed
forms: <u> = U, <u u> - <u>^2 = A^2/2, Favre stresses equal the Reynolds
ones (uniform density), <p> = p, and the temperature follows from p."""
import numpy as np

import oracle
import problems as P


def test_stats_closed_form():
    pr = P.small_channel(12, 10, 16)
    nz, ny, nx = pr.nz, pr.ny, pr.nx
    z = np.arange(nz) * (pr.lz / nz)
    y = np.asarray(pr.y)
    U = 1.0 + 0.3 * y
    A, m = 0.2, 3
    u = U[None, :, None] + A * np.sin(2 * np.pi * m * z / pr.lz)[:, None, None]
    u = np.broadcast_to(u, (nz, ny, nx))
    rho = np.full((nz, ny, nx), 1.3)
    p = np.full((nz, ny, nx), pr.R_gas * 1.1)
    zeros = np.zeros((nz, ny, nx))
    w = P.conserved_from_primitive(rho, u, zeros, zeros, p, pr.gamma)
    acc = oracle.stats(pr, w)
    mean = acc / nz
    names = oracle.STAT_NAMES
    g = {k: mean[i] for i, k in enumerate(names)}
    np.testing.assert_allclose(g["u"], np.broadcast_to(U[:, None], (ny, nx)), rtol=1e-13)
    np.testing.assert_allclose(g["uu"] - g["u"] ** 2, A * A / 2, rtol=1e-10)
    uf = g["rho_u"] / g["rho"]
    np.testing.assert_allclose(g["rho_uu"] / g["rho"] - uf ** 2, A * A / 2, rtol=1e-10)
    np.testing.assert_allclose(g["rho_uv"], 0.0, atol=1e-14)
    np.testing.assert_allclose(g["p"], pr.R_gas * 1.1, rtol=1e-12)
    np.testing.assert_allclose(g["pp"] - g["p"] ** 2, 0.0, atol=1e-14)
    np.testing.assert_allclose(g["T"], 1.1 / 1.3, rtol=1e-12)
    np.testing.assert_allclose(g["rho_rho"], 1.3 ** 2, rtol=1e-13)
    # accumulation adds
    acc2 = oracle.stats(pr, w, acc.copy())
    np.testing.assert_allclose(acc2, 2 * acc, rtol=1e-15)


def test_stats_means_closed_form_with_density_fluctuations():
    """Favre and Reynolds means differ when density and velocity fluctuate
    together: rho = r0 (1 + b s), u = U + a s, v = c s with s = sin(2 pi m z /
    L_z) over full periods (mean of s 0, of s^2 1/2, of s^3 0), uniform p.
    Then <rho> = r0, Favre u~ = U + a b/2, R11 = <rho u u>/<rho> - u~^2 =
    a^2 (1/2 - b^2/4), R12 = a c (1/2 - b^2/4), u_rms = a/sqrt 2, rho_rms =
    r0 b/sqrt 2, p_rms = 0; the x average of x-independent fields equals
    the field."""
    pr = P.small_channel(12, 10, 16)
    nz, ny, nx = pr.nz, pr.ny, pr.nx
    z = np.arange(nz) * (pr.lz / nz)
    s = np.sin(2 * np.pi * 2 * z / pr.lz)[:, None, None] * np.ones((nz, ny, nx))
    r0, b, a, c, U = 1.2, 0.3, 0.25, -0.1, 0.8
    rho = r0 * (1 + b * s)
    u = U + a * s
    v = c * s
    p = np.full((nz, ny, nx), pr.R_gas)
    w = P.conserved_from_primitive(rho, u, v, np.zeros_like(u), p, pr.gamma)
    acc = oracle.stats(pr, w)
    acc = oracle.stats(pr, w, acc)            # two samples of the same state
    for avg in (False, True):
        mn = oracle.stats_means(pr, acc, 2, average_x=avg)
        f = 1.0 / 2 - b * b / 4
        checks = {"rho": r0, "u_favre": U + a * b / 2, "v_favre": c * b / 2, "R11": a * a * f,
                  "R22": c * c * f, "R12": a * c * f, "R33": 0.0, "u": U,
                  "u_rms": a / np.sqrt(2), "rho_rms": r0 * b / np.sqrt(2), "p": pr.R_gas}
        for k, v_ in checks.items():
            np.testing.assert_allclose(mn[k], v_, rtol=1e-12, atol=1e-12, err_msg=k)
        # a zero variance from the difference of second moments: sqrt of rounding
        assert np.abs(mn["p_rms"]).max() <= 1e-7 * pr.R_gas
        assert mn["rho"].shape == ((ny,) if avg else (ny, nx))
    # T = p/(rho R): rho T = p/R is uniform, so the Favre mean of T is 1/r0
    mn = oracle.stats_means(pr, acc, 2)
    np.testing.assert_allclose(mn["T_favre"], 1.0 / r0, rtol=1e-12)
