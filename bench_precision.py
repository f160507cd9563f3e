#!/usr/bin/env python3
"""Precision-mode benchmark: FP32 fluxes against the FP64 path.

Workload: the compressible channel at 512x256x256 (33.5 M points; same
domain, physics and seeded initial field recipe as the 256x128x128
benchmark).  Both precisions advance 100 RK3 steps from the same state
with the same fixed time step (the CFL-0.8 step of the initial field), as
HIP-graph replays.  Prints one JSON line with the throughput of each
precision, the speedup, and per field (rho, rho u, rho v, rho w, rho E and
the derived u, T, p) the relative L-infinity and L2 differences of the
FP32-flux state from the FP64 state.  The comparison of both precisions
with the FP64 oracle after 100 steps is done by GPU tests: at 256x128x128
over the whole field (tests/test_gpu_configs.py::
test_full_size_channel_100_steps, the oracle taking about two minutes of
host time), and at this size on 1,024 seeded sample nodes against the
oracle's reference values, written once by
tests/golden/make_precision_samples.py (about 80 minutes on 8 host
threads; test_precision_mode_at_its_size_against_oracle_samples).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--nz", type=int, default=256)
    args = ap.parse_args()

    import numpy as np
    import torch

    import problems as P
    from paper_2004_02276_amd import Solver

    assert torch.cuda.is_available(), "bench_precision.py needs a GPU"
    pr = P.channel(args.nx, args.ny, args.nz)
    print(f"# {pr.name}: {pr.npts} points", file=sys.stderr, flush=True)
    # fixed time step: the CFL step of the initial field
    s = Solver(pr)
    s.advance(1, cfl=pr.cfl)
    dt = s.diagnostics()["dt"]
    s.close()
    out = {"metric": "FP32-flux vs FP64 state differences and speedup", "workload": pr.name,
           "points": pr.npts, "steps": args.steps, "dt": dt}
    states = {}
    for name, prec in (("fp64", 0), ("fp32flux", 1)):
        s = Solver(pr, precision=prec)
        s.advance(2, dt_fixed=dt)  # graph capture and warm-up
        s.set_state(pr.w0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(args.steps, dt_fixed=dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        states[name] = s.get_state()
        s.close()
        out[name] = {"mpoint_steps_per_s": pr.npts * args.steps / el / 1e6,
                     "ms_per_step": el * 1e3 / args.steps}
        print(f"# {name}: {out[name]}", file=sys.stderr, flush=True)
    out["speedup"] = out["fp32flux"]["mpoint_steps_per_s"] / out["fp64"]["mpoint_steps_per_s"]

    g = pr.gamma
    cv = pr.R_gas / (g - 1.0)

    def derived(w):
        r = w[0]
        u = w[1] / r
        ke = 0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / r ** 2
        T = (w[4] / r - ke) / cv
        return {"u": u, "T": T, "p": r * pr.R_gas * T}

    a, b = states["fp32flux"], states["fp64"]
    errs = {}
    for m, nm in enumerate(["rho", "rho_u", "rho_v", "rho_w", "rho_E"]):
        d = a[m] - b[m]
        errs[nm] = {"linf_rel": float(np.abs(d).max() / np.abs(b[m]).max()),
                    "l2_rel": float(np.linalg.norm(d) / np.linalg.norm(b[m]))}
    da, db = derived(a), derived(b)
    for nm in ("u", "T", "p"):
        d = da[nm] - db[nm]
        errs[nm] = {"linf_rel": float(np.abs(d).max() / np.abs(db[nm]).max()),
                    "l2_rel": float(np.linalg.norm(d) / np.linalg.norm(db[nm]))}
    out["fp32flux_vs_fp64"] = errs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
