"""GPU tests of the batched runner and the continuous-batching server.

Each instance's result must be the same alone and in the mix: the batched
persistent kernels process an instance with exactly its single-instance
arithmetic (same tiles, same reduction slots), so equality is bitwise.
"""
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def small_requests():
    return [
        P.request_problem(P.RequestSpec(0, 0.0, "turbulence", 24, 0.7, 900.0, 11, 6)),
        P.request_problem(P.RequestSpec(1, 0.0, "channel", 20, 1.5, 2000.0, 12, 6)),
        P.request_problem(P.RequestSpec(2, 0.0, "turbulence", 34, 2.5, 3000.0, 13, 6)),
        P.request_problem(P.RequestSpec(3, 0.0, "channel", 28, 0.4, 700.0, 14, 6)),
    ]


def test_batch_alone_equals_mix(gpu):
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd.serve import Batch
    prs = small_requests()
    say("[batch] solo runs")
    solo = []
    for pr in prs:
        s = Solver(pr, tiling=(64, 4, 8))
        s.advance(6, cfl=0.8)
        solo.append(s.get_state())
        s.close()
    say("[batch] mixed run with staggered admission")
    b = Batch(8)
    sv = [Solver(pr, tiling=(64, 4, 8)) for pr in prs]
    slots = {0: b.attach(sv[0]), 1: b.attach(sv[1])}
    done = {0: 0, 1: 0}
    for it in range(14):
        if it == 2:
            slots[2] = b.attach(sv[2]); done[2] = 0
        if it == 4:
            slots[3] = b.attach(sv[3]); done[3] = 0
        if not slots:
            break
        b.step(1)
        for k in list(slots):
            done[k] += 1
            if done[k] == 6:
                b.detach(slots.pop(k))
    gpu.cuda.synchronize()
    for k, s in enumerate(sv):
        w = s.get_state()
        say(f"    instance {k}: max |mix - alone| = {np.abs(w - solo[k]).max():.3e}")
        assert np.array_equal(w, solo[k])
        s.close()
    b.close()


def test_batch_matches_oracle(gpu):
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd.serve import Batch
    prs = small_requests()[:2]
    say("[batch] vs oracle")
    b = Batch(4)
    sv = [Solver(pr) for pr in prs]
    dts = [oracle.dt(pr) for pr in prs]
    for s, dt in zip(sv, dts):
        b.attach(s, dt_fixed=dt)
    b.step(5)
    for s, pr, dt in zip(sv, prs, dts):
        w_o = oracle.advance(pr, 5, dt_fixed=dt)
        w_g = s.get_state()
        err = max(np.abs(w_g[m] - w_o[m]).max() / np.abs(w_o[m]).max() for m in range(5))
        say(f"    {pr.name}: state error {err:.2e}")
        assert err <= 1e-10
        s.close()
    b.close()


def test_server_admission_and_results(gpu):
    from paper_2004_02276_amd.serve import Server, footprint_bytes
    # all six arrive at once; the budget fits roughly two of the larger
    # instances and less than the six together, so admissions must wait
    specs = [P.RequestSpec(i, 0.0, "turbulence" if i % 2 else "channel",
                           16 + 4 * i, 0.5 + 0.3 * i, 1000.0 + 200 * i, 40 + i, 8)
             for i in range(6)]
    prbs = {s.rid: P.request_problem(s) for s in specs}
    budget = int(2.2 * max(footprint_bytes(p) for p in prbs.values()))
    assert sum(footprint_bytes(p) for p in prbs.values()) > budget
    say(f"[server] budget {budget / 1e6:.1f} MB")
    srv = Server(P.request_problem, budget, max_slots=8, keep_states=True)
    rep = srv.run(specs, mode="batch", prebuilt=prbs)
    say(f"    batch: makespan {rep['makespan_s']:.2f}s p50 {rep['p50_step_ms']:.2f} ms "
        f"p99 {rep['p99_step_ms']:.2f} ms completed {rep['completed']}")
    assert rep["completed"] == len(specs)
    ser = Server(P.request_problem, budget, max_slots=8, keep_states=True)
    rep_s = ser.run(specs, mode="serial", prebuilt=prbs)
    assert rep_s["completed"] == len(specs)
    for rid in rep["results"]:
        a = rep["results"][rid].state
        b = rep_s["results"][rid].state
        assert np.array_equal(a, b), rid
    # the budget bounded the resident set: its peak stayed within the budget
    # and requests that arrived while it was full waited to be admitted
    say(f"    peak resident {rep['peak_resident_bytes'] / 1e6:.1f} MB, "
        f"{rep['waited_for_memory']} waited for memory")
    assert 0 < rep["peak_resident_bytes"] <= budget
    assert rep["waited_for_memory"] >= 1
    waited = [r for r in rep["results"].values() if r.admitted > r.arrival + 1e-4]
    assert len(waited) >= rep["waited_for_memory"]


def test_failed_request_is_retired_alone(gpu):
    """One request starts from a state with a negative-energy point: it
    goes non-physical, is stepped to its end with the others and retires
    'failed:' with its device status set, while the requests resident with
    it finish with states bit for bit equal to their runs alone."""
    from paper_2004_02276_amd import Solver
    from paper_2004_02276_amd.serve import Server
    specs = [P.RequestSpec(i, 0.0, "turbulence" if i % 2 else "channel", 16 + 4 * i,
                           0.5 + 0.3 * i, 1000.0 + 200 * i, 30 + i, 12) for i in range(3)]
    prbs = {s.rid: P.request_problem(s) for s in specs}
    w_bad = prbs[1].w0.copy()
    w_bad[4, 2, 3, 4] = -1.0
    prbs[1] = P.with_state(prbs[1], w_bad)
    say("[server] failure isolation")
    rep = Server(P.request_problem, 1 << 34, max_slots=8, keep_states=True).run(
        specs, mode="batch", prebuilt=prbs)
    assert rep["results"][1].status.startswith("failed"), rep["results"][1].status
    assert rep["failed"] == 1 and rep["completed"] == 2
    for rid in (0, 2):
        s = Solver(prbs[rid], tiling=(64, 4, 16))   # the server's tiling
        s.advance(specs[rid].nsteps, cfl=prbs[rid].cfl)
        alone = s.get_state()
        s.close()
        assert np.array_equal(rep["results"][rid].state, alone), rid


def test_multi_step_replays_equal_single_steps(gpu):
    """Replaying several batch steps between host checks gives the same
    states as one step per check."""
    from paper_2004_02276_amd.serve import Server
    specs = [P.RequestSpec(i, 0.0, "turbulence" if i % 2 else "channel", 16 + 4 * i,
                           0.5 + 0.3 * i, 1000.0 + 200 * i, 20 + 3 * i, 13) for i in range(3)]
    prbs = {s.rid: P.request_problem(s) for s in specs}
    say("[server] chunked replays")
    out = []
    for chunk in (1, 8):
        rep = Server(P.request_problem, 1 << 34, max_slots=8, keep_states=True,
                     max_chunk=chunk).run(specs, mode="batch", prebuilt=prbs)
        assert rep["completed"] == 3 and rep["max_chunk"] == chunk
        assert all(r.steps == sp.nsteps for r, sp in zip(rep["results"].values(), specs))
        out.append(rep["results"])
    for rid in out[0]:
        assert np.array_equal(out[0][rid].state, out[1][rid].state), rid


def test_autotuner_keeps_the_fastest_step(gpu):
    """The tuner ranks (tile, kz) by the per-step time of the phases the
    tiling changes and keeps the minimum; the lookup returns it."""
    from paper_2004_02276_amd import autotune
    pr = P.small_channel(48, 24, 16)
    say("[autotune]")
    res = autotune.tune(pr, steps=2, tiles=[(64, 4), (32, 8)], kzs=[4, 16], save=False)
    assert set(res["all"]) == {"64x4/kz4", "64x4/kz16", "32x8/kz4", "32x8/kz16"}
    best = min(res["all"], key=res["all"].get)
    assert res["ms"] == res["all"][best] and f"{res['tile'][0]}x{res['tile'][1]}/kz{res['kz']}" == best
    assert all(v > 0 for v in res["all"].values())
    ph = {"rhs": (0.5, 3), "rk": (0.1, 3), "force": (0.01, 3), "weno": (9.0, 3)}
    assert abs(autotune.step_ms(ph, 1) - 1.83) < 1e-12   # weno does not depend on the tile


def test_server_rejects_unbatchable_configurations(gpu):
    """A request the batched kernels do not run (here sixth-order central
    and seventh-order WENO) is rejected with a status in batch mode while
    the others complete; the serial loop runs all of them."""
    import dataclasses
    from paper_2004_02276_amd.serve import Server
    specs = [P.RequestSpec(i, 0.0, "turbulence" if i % 2 else "channel", 16 + 4 * i,
                           0.5 + 0.3 * i, 1000.0 + 200 * i, 20, 8) for i in range(3)]
    prbs = {s.rid: P.request_problem(s) for s in specs}
    prbs[1] = dataclasses.replace(prbs[1], central_order=6, weno_order=7)
    say("[server] unbatchable request")
    rep = Server(P.request_problem, 1 << 34, max_slots=8).run(specs, mode="batch", prebuilt=prbs)
    assert rep["completed"] == 2 and rep["rejected"] == 1
    assert rep["results"][1].status == "rejected: configuration not batchable"
    rep_s = Server(P.request_problem, 1 << 34, max_slots=8).run(specs, mode="serial", prebuilt=prbs)
    assert rep_s["completed"] == 3
