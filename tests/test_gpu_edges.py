"""GPU parity at the edges of the input space: the smallest grids the
library accepts (4 nodes along an axis, tiles far larger than the grid),
odd sizes, a hybrid sensor that flags nothing (empty interface lists) or
everything, and the degenerate uniform state, whose right-hand side is
zero up to the rounding of the difference weights."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import problems as P

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
STATE_TOL = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    return torch


def field_errors(a, b):
    scale_all = max(np.abs(b).max(), 1e-300)
    out = []
    for m in range(5):
        s = np.abs(b[m]).max()
        if s < 1e-12 * scale_all:
            s = scale_all
        out.append(float(np.abs(a[m] - b[m]).max() / s))
    return out


def _random_periodic(nx, ny, nz, seed, mach=0.8, sensor_mode=P.SENSOR_HYBRID, theta_star=0.1):
    """A periodic box of nx x ny x nz nodes with a smooth random state
    (density, velocity and pressure perturbations of a few low modes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = P.decaying_turbulence(8, mach=mach, re=600.0, seed=seed)
    L = 2 * np.pi
    x = np.arange(nx) * (L / nx)
    y = np.arange(ny) * (L / ny)
    z = np.arange(nz) * (L / nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")

    def field(amp):
        a = rng.uniform(-1, 1, size=6)
        return amp * (a[0] * np.sin(X + a[1]) + a[2] * np.cos(Y + a[3]) + a[4] * np.sin(Z + a[5]))

    rho = 1.0 + field(0.1)
    u, v, w = field(0.5), field(0.5), field(0.5)
    p = base.R_gas * (1.0 + field(0.1))
    w0 = P.conserved_from_primitive(rho, u, v, w, p, base.gamma)
    yy, ye, yee = P.uniform_periodic_y(ny, L)
    return P.with_state(base, w0, nx=nx, ny=ny, nz=nz, y=yy, y_eta=ye, y_etaeta=yee, lx=L, lz=L,
                        sensor_mode=sensor_mode, theta_star=theta_star)


EDGE_CASES = {
    # smallest accepted grid, every direction periodic, hybrid sensor
    "periodic_4x4x4": lambda: _random_periodic(4, 4, 4, 21),
    # odd sizes, none a multiple of a tile or of the flag kernel's 16 nodes
    "periodic_5x7x9": lambda: _random_periodic(5, 7, 9, 22),
    "periodic_67x5x4_weno_all": lambda: _random_periodic(67, 5, 4, 23,
                                                          sensor_mode=P.SENSOR_WENO_ALL),
    # walls with the fewest nodes between them
    "channel_4x4x4": lambda: P.small_channel(4, 4, 4),
    "channel_9x5x6": lambda: P.small_channel(9, 5, 6),
    # inflow, outflow and imposed shock on a short box
    "sbli_8x6x4": lambda: P.small_sbli(8, 6, 4, theta_star=0.02),
    # hybrid sensor that flags no node: empty interface lists
    "no_flagged_node": lambda: _random_periodic(24, 16, 12, 24, theta_star=2.0),
    # hybrid sensor that flags every compressing node
    "every_compression_flagged": lambda: _random_periodic(24, 16, 12, 25, theta_star=0.0),
}


@pytest.mark.parametrize("case", list(EDGE_CASES))
def test_edge_case_rhs_and_steps(torch_cuda, case):
    from paper_2004_02276_amd import Solver
    pr = EDGE_CASES[case]()
    say(f"[edge] {case} {pr.nx}x{pr.ny}x{pr.nz} sensor mode {pr.sensor_mode}")
    r_o, th_o, nf_o, if_o, _ = oracle.rhs(pr, want_flags=True)
    s = Solver(pr)
    r_g = s.rhs().cpu().numpy()
    _, nf_g, if_g = s.export_sensor()
    d = s.diagnostics()
    if pr.sensor_mode > 0:
        assert np.array_equal(if_g.cpu().numpy(), if_o)
    if pr.sensor_mode == P.SENSOR_HYBRID:
        assert np.array_equal(nf_g.cpu().numpy(), nf_o)
    if case == "no_flagged_node":
        assert not nf_o.any() and not if_o.any() and d["weno_frac"] == [0.0, 0.0, 0.0]
    errs = field_errors(r_g, r_o)
    say(f"    rhs errors {['%.1e' % e for e in errs]}  weno share {d['weno_frac']}")
    assert max(errs) <= RHS_TOL, errs
    dt = oracle.dt(pr)
    s.advance(10, dt_fixed=dt)
    w_g = s.get_state()
    s.close()
    w_o = oracle.advance(pr, 10, dt_fixed=dt)
    errs = field_errors(w_g, w_o)
    say(f"    10-step state errors {['%.1e' % e for e in errs]}")
    assert max(errs) <= STATE_TOL, errs


@pytest.mark.parametrize("mode", [P.SENSOR_OFF, P.SENSOR_HYBRID, P.SENSOR_WENO_ALL])
def test_uniform_state_has_zero_rhs(torch_cuda, mode):
    """A uniform state at rest between isothermal walls at its own
    temperature, and a uniform moving state in a periodic box: every flux
    difference and derivative vanishes, up to the rounding of the
    difference weights (their sums vanish only in exact arithmetic), far
    below 1e-12 of the pressure-gradient scale p/dx on both sides."""
    from paper_2004_02276_amd import Solver
    say(f"[uniform] sensor mode {mode}")
    ch = P.small_channel(24, 12, 8)
    shape = (ch.nz, ch.ny, ch.nx)
    rest = P.conserved_from_primitive(np.ones(shape), np.zeros(shape), np.zeros(shape),
                                      np.zeros(shape), np.full(shape, ch.R_gas), ch.gamma)
    bcs = list(ch.bcs)
    bcs[P.FACE_YM] = (P.BC_WALL_ISOTHERMAL, np.array([1.0]))
    bcs[P.FACE_YP] = (P.BC_WALL_ISOTHERMAL, np.array([1.0]))
    walls = dataclasses.replace(P.with_state(ch, rest), bcs=bcs, forcing=False, sensor_mode=mode)
    box = _random_periodic(16, 12, 8, 26, sensor_mode=mode)
    moving = P.conserved_from_primitive(np.full((8, 12, 16), 1.3), np.full((8, 12, 16), 0.4),
                                        np.full((8, 12, 16), -0.2), np.full((8, 12, 16), 0.1),
                                        np.full((8, 12, 16), box.R_gas), box.gamma)
    for pr in (walls, P.with_state(box, moving)):
        s = Solver(pr)
        r_g = s.rhs().cpu().numpy()
        s.close()
        r_o = oracle.rhs(pr)
        scale = pr.R_gas / min(pr.dx, pr.dz, float(np.min(pr.y_eta)) / pr.ny)
        say(f"    max |R| gpu {np.abs(r_g).max():.1e} oracle {np.abs(r_o).max():.1e} "
            f"(p/dx {scale:.1e})")
        assert np.abs(r_o).max() <= 1e-12 * scale
        assert np.abs(r_g).max() <= 1e-12 * scale


def test_time_step_same_from_sensor_and_from_its_own_pass(torch_cuda):
    """The CFL time step equals the oracle's, and is the same bit for bit
    whether the first stage's sensor reduces the bounds (hybrid sensor) or
    the separate reduction does (shock capturing everywhere, sensor off):
    both evaluate every node's bound with the same arithmetic and take
    exact maxima."""
    from paper_2004_02276_amd import Solver
    say("[dt paths]")
    for make in (lambda m: P.decaying_turbulence(24, mach=0.5, re=800.0, seed=11, sensor_mode=m),
                 lambda m: dataclasses.replace(P.small_channel(24, 20, 12), sensor_mode=m)):
        dts = []
        for mode in (P.SENSOR_HYBRID, P.SENSOR_WENO_ALL, P.SENSOR_OFF):
            pr = make(mode)
            s = Solver(pr)
            s.rk_step(cfl=0.8)
            dts.append(s.diagnostics()["dt"])
            s.close()
        dt_o = oracle.dt(pr, cfl=0.8)
        say(f"    {pr.name}: gpu {dts[0]:.17e} oracle {dt_o:.17e}")
        assert dts[0] == dts[1] == dts[2], dts
        assert abs(dts[0] - dt_o) <= 1e-12 * dt_o
