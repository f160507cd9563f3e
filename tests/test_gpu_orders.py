"""GPU parity of the scheme-order variants (central flux and viscous terms of
order 2 and 6, WENO of order 3 and 7) against the FP64 oracle, through the
C ABI, with the tolerances of the default scheme: right-hand side within
1e-12 and state within 1e-10 per conserved field (relative L-infinity),
sensor values within 1e-13 and flag masks exact.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import problems as P
from tests.test_gpu_parity import (RHS_TOL, STATE_TOL, _tgv_ragged, field_errors, gpu_rhs, say,
                                   torch_cuda)  # noqa: F401

pytestmark = pytest.mark.gpu


def orders(pr, central, weno):
    return dataclasses.replace(pr, central_order=central, weno_order=weno)


def _dit(seed, mach=1.5, mode=P.SENSOR_HYBRID, viscous=True):
    pr = P.decaying_turbulence(24, mach=mach, re=800.0, seed=seed)
    return dataclasses.replace(pr, sensor_mode=mode, viscous=viscous)


RHS_CASES = {
    "tgv32_c2_w3": lambda: orders(P.taylor_green(32), 2, 3),
    "tgv32_c6_w5": lambda: orders(P.taylor_green(32), 6, 5),
    "tgv_ragged_c6": lambda: orders(_tgv_ragged(), 6, 5),
    "tgv_ragged_c2": lambda: orders(_tgv_ragged(), 2, 5),
    "dit24_hybrid_c6_w7": lambda: orders(_dit(11), 6, 7),
    "dit24_hybrid_c2_w3": lambda: orders(_dit(11), 2, 3),
    "dit24_hybrid_c4_w7": lambda: orders(_dit(15), 4, 7),
    "dit24_weno_all_w7": lambda: orders(_dit(12, 2.5, P.SENSOR_WENO_ALL), 6, 7),
    "dit24_weno_all_w3": lambda: orders(_dit(12, 2.5, P.SENSOR_WENO_ALL), 2, 3),
    "dit24_inviscid_c6_w7": lambda: orders(_dit(13, viscous=False), 6, 7),
    "dit24_inviscid_c2_w3": lambda: orders(_dit(13, viscous=False), 2, 3),
    "channel_24x20x12_c6_w7": lambda: orders(P.small_channel(24, 20, 12), 6, 7),
    "channel_70x22x10_c2_w3": lambda: orders(P.small_channel(70, 22, 10), 2, 3),
    "sbli_64x32x8_c6_w7": lambda: orders(P.small_sbli(64, 32, 8), 6, 7),
    "sbli_100x36x6_c6_w3": lambda: orders(P.small_sbli(100, 36, 6, theta_star=0.02), 6, 3),
    "sbli_64x32x8_c2_w7": lambda: orders(P.small_sbli(64, 32, 8), 2, 7),
    "bl_48x32x16_c6_w7": lambda: orders(P.small_boundary_layer(), 6, 7),
}


@pytest.mark.parametrize("case", list(RHS_CASES))
def test_rhs_parity_orders(torch_cuda, case):
    pr = RHS_CASES[case]()
    say(f"[rhs parity orders] {case} {pr.nx}x{pr.ny}x{pr.nz} mode={pr.sensor_mode}")
    r_o, th_o, nf_o, if_o, _ = oracle.rhs(pr, want_flags=True)
    r_g, th_g, nf_g, if_g = gpu_rhs(pr)
    if pr.sensor_mode == P.SENSOR_HYBRID:
        assert np.abs(th_g - th_o).max() <= 1e-13, "sensor values differ"
        assert (nf_g == nf_o).all(), "node flags differ"
    if pr.sensor_mode > 0:
        assert (if_g == if_o).all(), "interface flags differ"
    errs = field_errors(r_g, r_o)
    say(f"    errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= RHS_TOL, errs


@pytest.mark.parametrize("case", ["dit24_hybrid_c6_w7", "dit24_weno_all_w3", "sbli_64x32x8_c2_w7"])
def test_weno_interface_fluxes_orders(torch_cuda, case):
    """Shock-capturing interface fluxes at every flagged interface within
    1e-12 of the oracle's (the right-hand-side bar): the WENO7 smoothness
    indicators are quadratic forms with cancelling coefficients up to
    17246/240, so their rounding is about 40 times that of WENO5's, and
    the two sides evaluate them in different orders."""
    from paper_2004_02276_amd import Solver
    pr = RHS_CASES[case]()
    say(f"[iface flux orders] {case}")
    s = Solver(pr)
    s.rhs(s.state)
    ifl = s.export_sensor()[2].cpu().numpy()
    fg = [s.export_iface_flux(d).cpu().numpy() for d in range(3)]
    s.close()
    for d in range(3):
        mask = ((ifl >> d) & 1).astype(bool)
        assert mask.any()
        fo = oracle.iface_flux(pr, d)
        for m in range(5):
            scale = max(np.abs(fo[m][mask]).max(), 1e-300)
            err = np.abs(fg[d][m][mask] - fo[m][mask]).max() / scale
            assert err <= RHS_TOL, (d, m, err)


STEP_CASES = {
    "channel_24x20x12_c6_w7_60steps": (lambda: orders(P.small_channel(24, 20, 12), 6, 7), 60, True),
    "sbli_64x32x8_c2_w3_60steps": (lambda: orders(P.small_sbli(64, 32, 8), 2, 3), 60, True),
    "dit24_hybrid_c6_w7_30steps": (lambda: orders(_dit(11, mach=0.5), 6, 7), 30, False),
    "bl_48x32x16_c6_w7_20steps": (lambda: orders(P.small_boundary_layer(), 6, 7), 20, False),
}


@pytest.mark.parametrize("case", list(STEP_CASES))
def test_state_parity_orders(torch_cuda, case):
    from paper_2004_02276_amd import Solver
    make, nsteps, fixed = STEP_CASES[case]
    pr = make()
    say(f"[state parity orders] {case}")
    dt_fixed = oracle.dt(pr) if fixed else 0.0
    w_o = oracle.advance(pr, nsteps, dt_fixed=dt_fixed)
    s = Solver(pr)
    s.advance(nsteps, cfl=pr.cfl, dt_fixed=dt_fixed)
    w_g = s.get_state()
    d = s.diagnostics()
    s.close()
    errs = field_errors(w_g, w_o)
    say(f"    errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= STATE_TOL, errs
    assert d["step"] == nsteps


def test_viscous_time_step_bound_follows_the_order(torch_cuda):
    """The CFL time step of a viscous case equals the oracle's for each
    central order (the viscous bound uses the order's second-derivative
    radius)."""
    from paper_2004_02276_amd import Solver
    base = P.small_channel(24, 20, 12)
    say("[dt orders]")
    for co in (2, 4, 6):
        pr = dataclasses.replace(base, central_order=co, mu_ref=base.mu_ref * 50.0)
        s = Solver(pr)
        s.rk_step(cfl=0.5)
        dt_g = s.diagnostics()["dt"]
        s.close()
        dt_o = oracle.dt(pr, cfl=0.5)
        assert abs(dt_g - dt_o) <= 1e-12 * dt_o, (co, dt_g, dt_o)


def test_full_size_channel_rhs_c6_w7(torch_cuda):
    pr = orders(P.channel(), 6, 7)
    say(f"[full orders] channel {pr.nx}x{pr.ny}x{pr.nz} c6 w7")
    r_o, th_o, nf_o, if_o, _ = oracle.rhs(pr, want_flags=True)
    r_g, th_g, nf_g, if_g = gpu_rhs(pr)
    assert np.abs(th_g - th_o).max() <= 1e-13
    assert (nf_g == nf_o).all() and (if_g == if_o).all()
    errs = field_errors(r_g, r_o)
    say(f"    errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= RHS_TOL, errs


def test_fp32_flux_mode_with_orders(torch_cuda):
    pr = orders(P.small_channel(24, 20, 12), 6, 7)
    say("[fp32 flux orders]")
    r_o = oracle.rhs(pr)
    r_g = gpu_rhs(pr, precision=1)[0]
    errs = field_errors(r_g, r_o)
    say(f"    fp32-flux RHS errors {['%.2e' % e for e in errs]}")
    assert max(errs) < 1e-3


def test_scheme_setter_errors(torch_cuda):
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd import _binding as B
    from paper_2004_02276_amd.serve import Batch
    say("[scheme setter errors]")
    s = Solver(P.taylor_green(16))
    for co, wo in ((8, 5), (4, 9), (3, 5), (4, 4)):
        with pytest.raises(B.CdnsError) as err:
            s.set_scheme(co, wo)
        assert err.value.status == B.CDNS_EINVAL
    s.set_scheme(6, 7)
    with pytest.raises(B.CdnsError) as err:
        s.set_tiling(32, 8, 4)
    assert err.value.status == B.CDNS_EUNSUP
    s.set_tiling(64, 4, 8)
    b = Batch(4)
    with pytest.raises(B.CdnsError) as err:
        b.attach(s)
    assert err.value.status == B.CDNS_EUNSUP
    b.close()
    s.close()
    # the sixth-order z stencil needs nz >= 6
    thin = dataclasses.replace(P.small_sbli(64, 32, 4), central_order=6)
    with pytest.raises(B.CdnsError) as err:
        Solver(thin)
    assert err.value.status == B.CDNS_EINVAL
