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
