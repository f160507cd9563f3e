"""The no-allocation diagnostics entry point (cdns_diagnostics_noalloc)
against cdns_diagnostics on the same states: two calls in a row, the
second on a smaller grid (fewer partial-sum blocks than the first, whose
partials stay in the shared scratch array), an explicit state argument,
and the size limit."""
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

U = 2.0 ** -53


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


def _compare(pr, s, out, w):
    """Sums within the rounding bound of two summation orders of the same N
    terms (2 (N - 1) u sum |x_i dV_i|); extrema and counts identical."""
    d = s.diagnostics()
    ref = np.array([d["mass"]] + list(d["mom"]) + [d["energy"], d["kinetic"], d["rho_min"],
                    d["p_min"], d["mach_max"], float(d["nonfinite"])])
    g = out.cpu().numpy()
    n = w[0].size
    dv = pr.dx * pr.dz * (1.0 / pr.ny) * np.asarray(pr.y_eta)[None, :, None]
    mags = [np.sum(np.abs(w[m]) * dv) for m in range(5)]
    mags.append(np.sum(0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / w[0] * dv))
    bound = 2.0 * (n - 1) * U * np.array(mags)
    err = np.abs(g[:6] - ref[:6])
    say(f"    sums |diff| {['%.1e' % e for e in err]}  bound {['%.1e' % b for b in bound]}")
    assert np.all(err <= bound), (err, bound)
    assert np.array_equal(g[6:], ref[6:]), (g[6:], ref[6:])


def test_noalloc_diagnostics_match_diagnostics(torch_cuda):
    from paper_2004_02276_amd import Solver
    t = torch_cuda
    big = P.small_sbli(128, 64, 16)      # 131,072 points: 32 partial blocks
    small = P.small_channel(24, 20, 12)  # 5,760 points: 2 partial blocks
    for pr in (big, small):
        say(f"[noalloc diagnostics] {pr.name} {pr.nx}x{pr.ny}x{pr.nz}")
        s = Solver(pr)
        s.advance(3, dt_fixed=oracle.dt(pr))
        out = t.full((12,), -7.0, dtype=t.float64, device=s.device)
        s.diagnostics_noalloc(out=out)
        w = s.get_state()
        _compare(pr, s, out[:10], w)
        assert out[10].item() == -7.0 and out[11].item() == -7.0  # nothing written past the slots
        # an explicit state argument: the initial state
        w0 = t.from_numpy(np.ascontiguousarray(pr.w0)).to(s.device)
        out2 = s.diagnostics_noalloc(w=w0)
        s.set_state(pr.w0)
        _compare(pr, s, out2, pr.w0)
        s.close()


def test_noalloc_diagnostics_rejects_grids_beyond_the_maximum(torch_cuda):
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd import _binding as B
    pr0 = P.taylor_green(8)
    nx, ny, nz = 1024, 256, 129                     # 33,816,576 points > 2^25
    assert nx * ny * nz > B.NOALLOC_MAX_POINTS
    y, ye, yee = P.uniform_periodic_y(ny, 1.0)
    pr = dataclasses.replace(pr0, w0=None, nx=nx, ny=ny, nz=nz, y=y, y_eta=ye, y_etaeta=yee, lx=1.0, lz=1.0)
    s = Solver(pr)
    with pytest.raises(B.CdnsError) as err:
        s.diagnostics_noalloc()
    assert err.value.status == B.CDNS_EINVAL and "maximum" in str(err.value)
    s.close()
