"""State copies and the sensor-mask hooks of the C ABI (cdns_set_state,
cdns_get_state, cdns_export_flags, cdns_import_flags) on the GPU."""
import dataclasses

import numpy as np
import pytest

import oracle
import problems as P
from tests.test_gpu_parity import RHS_TOL, field_errors, say, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def test_state_copies_round_trip(torch_cuda):
    from paper_2004_02276_amd import Solver
    pr = P.small_channel(24, 20, 12)
    say("[state copies]")
    s = Solver(pr)
    assert np.array_equal(s.get_state(), pr.w0)  # host upload at creation
    w2 = pr.w0 * 1.01
    s.set_state(w2)                               # from host
    assert np.array_equal(s.get_state(), w2)
    d = torch_cuda.from_numpy(pr.w0).to("cuda")
    s.set_state(d)                                # device to device
    assert np.array_equal(s.get_state(), pr.w0)
    s.close()


def test_flag_export_and_import(torch_cuda):
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd import _binding as B
    pr = P.decaying_turbulence(24, mach=1.5, re=800.0, seed=11)
    say("[flag hooks]")
    _, _, nf_o, _, _ = oracle.rhs(pr, want_flags=True)
    s = Solver(pr)
    r_ref = s.rhs(s.state).cpu().numpy()
    nf = s.export_flags().cpu().numpy()
    assert np.array_equal(nf, s.export_sensor()[1].cpu().numpy())
    assert np.array_equal(nf, nf_o)
    # the oracle's mask imported: the same right-hand side, bit for bit
    s.import_flags(nf_o)
    r_imp = s.rhs(s.state).cpu().numpy()
    assert np.array_equal(r_imp, r_ref)
    # every node flagged: the interface set of the WENO-everywhere mode
    s.import_flags(np.ones_like(nf_o))
    r_all = s.rhs(s.state).cpu().numpy()
    assert np.array_equal(s.export_flags().cpu().numpy(), np.ones_like(nf_o))
    # the import is used once: the next evaluation runs the sensor again
    assert np.array_equal(s.rhs(s.state).cpu().numpy(), r_ref)
    # a step drops a pending import (its sensor overwrites the node flags)
    w_start = s.get_state()
    s.import_flags(np.ones_like(nf_o))
    s.rk_step(dt_fixed=1e-4)
    s.rhs(s.state)
    nf_next = s.export_flags().cpu().numpy()
    _, _, nf_o2, _, _ = oracle.rhs(P.with_state(pr, s.get_state()), want_flags=True)
    assert np.array_equal(nf_next, nf_o2)
    s.set_state(w_start)
    s.close()
    pr2 = dataclasses.replace(pr, sensor_mode=P.SENSOR_WENO_ALL)
    s2 = Solver(pr2)
    r_mode2 = s2.rhs(s2.state).cpu().numpy()
    s2.close()
    assert np.array_equal(r_all, r_mode2)
    errs = field_errors(r_all, oracle.rhs(pr2))
    assert max(errs) <= RHS_TOL, errs
    # node flags are a hybrid-mode input only
    s3 = Solver(P.taylor_green(16))
    with pytest.raises(B.CdnsError) as err:
        s3.import_flags(np.zeros((16, 16, 16), np.uint8))
    assert err.value.status == B.CDNS_EINVAL
    s3.close()


def test_configuration_refused_while_batched(torch_cuda):
    """A batch runs an attached context from a snapshot of its descriptor,
    so boundary, tiling and scheme changes wait for the detach."""
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd import _binding as B
    from paper_2004_02276_amd.serve import Batch
    say("[batched configuration]")
    pr = P.small_channel(24, 20, 12)
    s = Solver(pr)
    b = Batch(4)
    slot = b.attach(s)
    for call in (lambda: s.set_scheme(6, 7), lambda: s.set_tiling(64, 4, 8),
                 lambda: B.check(s.lib, s.ctx, s.lib.cdns_set_bc(
                     s.ctx, 2, P.BC_WALL_ADIABATIC, None, 0), "cdns_set_bc")):
        with pytest.raises(B.CdnsError) as err:
            call()
        assert err.value.status == B.CDNS_EBUSY
    b.detach(slot)
    s.set_scheme(6, 7)
    b.close()
    s.close()


POISON_CASES = {
    "channel_forced": (lambda: P.small_channel(24, 20, 12), None),
    "channel_32x8": (lambda: P.small_channel(40, 20, 12), (32, 8, 4)),
    "sbli": (lambda: P.small_sbli(64, 32, 8), None),
    "boundary_layer": (lambda: P.small_boundary_layer(), None),
    "weno_everywhere": (lambda: P.with_state(P.decaying_turbulence(16, mach=0.8, re=800.0, seed=5),
                                             P.decaying_turbulence(16, mach=0.8, re=800.0,
                                                                   seed=5).w0,
                                             sensor_mode=P.SENSOR_WENO_ALL), None),
}


@pytest.mark.parametrize("case", list(POISON_CASES))
def test_nan_poisoned_workspace_gives_the_same_results(torch_cuda, case):
    """With every work region of the workspace filled with NaN before first
    use, a right-hand side, eager and graph-replayed steps give bit for bit
    the results of a fresh workspace: no kernel reads memory it has not
    written."""
    from paper_2004_02276_amd import Solver
    make, tiling = POISON_CASES[case]
    pr = make()
    say(f"[poisoned workspace] {case}")
    out = []
    for poison in (False, True):
        s = Solver(pr, tiling=tiling)
        if poison:
            s.poison_workspace()
            s.set_state(pr.w0)
        r = s.rhs().cpu().numpy()
        s.rk_step(cfl=pr.cfl)
        s.advance(6, cfl=pr.cfl)
        d = s.diagnostics()
        out.append((r, s.get_state(), d["dt"], d["mass"]))
        s.close()
    (r0, w0, dt0, m0), (r1, w1, dt1, m1) = out
    assert np.isfinite(r1).all() and np.isfinite(w1).all()
    assert np.array_equal(r0, r1) and np.array_equal(w0, w1)
    assert dt0 == dt1 and m0 == m1
