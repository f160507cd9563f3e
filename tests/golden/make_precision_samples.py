#!/usr/bin/env python3
"""Oracle reference samples of the precision-mode workload.

The compressible channel at 512x256x256 (33.5 M points, the benchmark's
domain, physics and seeded initial field) advanced 100 RK3 steps by the
FP64 oracle with the fixed time step of the initial field (the CFL-0.8
step), one step per call so that progress can be followed.  Written to
channel512x256x256_100steps_oracle.txt beside this script: the time step,
the largest magnitude over the whole domain of each conserved field and of
u, T and p (the denominators of the relative L-infinity errors), the
relative-L2 denominators sqrt(sum x^2) over the samples, and the final
state at 1,024 sample nodes drawn with a fixed seed.

Calls only the oracle.  About two hours on 8 host threads:

    python tests/golden/make_precision_samples.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

NX, NY, NZ, STEPS = 512, 256, 256, 100
NSAMP, SAMPLE_SEED = 1024, 4
OUT = os.path.join(HERE, "channel512x256x256_100steps_oracle.txt")


def derived(pr, w):
    """u, T and p of conserved states w [5, ...] (the caloric and thermal
    equations of state of the model)."""
    cv = pr.R_gas / (pr.gamma - 1.0)
    r = w[0]
    u = w[1] / r
    ke = 0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / r ** 2
    T = (w[4] / r - ke) / cv
    return np.stack([u, T, r * pr.R_gas * T])


def sample_nodes():
    """(k, j, i) of the sample nodes: distinct, drawn uniformly with a fixed seed."""
    rng = np.random.default_rng(SAMPLE_SEED)
    flat = np.sort(rng.choice(NX * NY * NZ, size=NSAMP, replace=False))
    k, rem = np.divmod(flat, NX * NY)
    j, i = np.divmod(rem, NX)
    return k, j, i


def main():
    import oracle
    import problems as P
    pr = P.channel(NX, NY, NZ)
    dt = oracle.dt(pr)
    print(f"{pr.name}: {pr.npts} points, dt {dt!r}, {oracle.num_threads()} threads", flush=True)
    w = pr.w0
    t0 = time.perf_counter()
    for s in range(STEPS):
        w = oracle.advance(pr, 1, w=w, dt_fixed=dt)
        print(f"step {s + 1}/{STEPS} {time.perf_counter() - t0:.0f} s", flush=True)
    w = w.reshape(5, NZ, NY, NX)
    d = derived(pr, w)
    wmax = np.abs(w).reshape(5, -1).max(axis=1)
    dmax = np.abs(d).reshape(3, -1).max(axis=1)
    k, j, i = sample_nodes()
    ws = w[:, k, j, i]
    ds = derived(pr, ws)
    l2w = np.sqrt((ws ** 2).sum(axis=1))
    l2d = np.sqrt((ds ** 2).sum(axis=1))
    with open(OUT, "w") as fh:
        fh.write("# Channel 512x256x256 (benchmark recipe), 100 RK3 steps of the FP64 oracle from\n"
                 "# the seeded initial field at the fixed CFL-0.8 time step of that field.\n"
                 "# Written by make_precision_samples.py (calls only the oracle).\n")
        fh.write(f"dt {dt!r}\nsteps {STEPS}\n")
        fh.write("max_abs " + " ".join(repr(float(x)) for x in np.concatenate([wmax, dmax])) + "\n")
        fh.write("l2_samples " + " ".join(repr(float(x)) for x in np.concatenate([l2w, l2d])) + "\n")
        fh.write("# k j i rho rho_u rho_v rho_w rho_E\n")
        for n in range(NSAMP):
            fh.write(f"{k[n]} {j[n]} {i[n]} " + " ".join(repr(float(x)) for x in ws[:, n]) + "\n")
    print(f"wrote {OUT} after {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
