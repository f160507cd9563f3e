#!/usr/bin/env python3
"""Throughput benchmark of the RK3 step of the compressible Navier-Stokes
solver on one MI355X.

Workload (default): the compressible channel 256x128x128 (4.19 M points,
FP64 state, isothermal staggered walls on a tanh-stretched grid, bulk Mach
1.5, Re_b = 3000, hybrid central/WENO with the Ducros sensor, bulk
forcing), synthetic seeded initial field.  --workload sbli (shock on a
boundary layer, 1024x256x128), tgv (32^3) and bl (spatially developing
boundary layer with digital-filter inflow, 1024x128x128) give reference
figures on the other configurations.  A step is one full RK3 step (three
stages of ghost planes, sensor, flag compaction, WENO on lists, fused
right-hand side, forcing reduction and update), replayed from a HIP graph.

Prints ONE JSON line with the throughput (Mpoint-RK-steps/s), the roofline
of the dominant kernel (durations from HIP events on the library's stream,
over a kernel-by-kernel replay of the same timed steps from the same
state) and the FP64 oracle timed on the host cores on a bounded sample of
the same workload.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoint-RK-steps/s (hybrid RHS) & % HBM peak; batched p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
# Algorithmic bytes per point: one RK3 step must read w and write w', R
# (stage 0), read w, R_prev and write w', R (stage 1), read w, R_prev and
# write w' (stage 2) = 400 B; the lazy bulk forcing adds one 8-byte field
# per stage written and read = 448 B with forcing.
STEP_BYTES_PER_PT = 400.0
STEP_BYTES_PER_PT_FORCED = 448.0
# The fused right-hand-side kernel must read w (40 B) and write R (40 B).
# Without bulk forcing it also does the stage's update: read w, write w', R
# (stage 0), read w, R_prev and write w', R (stage 1), read w, R_prev and
# write w' (stage 2), a mean of 400 / 3 B per point and stage.  With bulk
# forcing it writes R (the force is reduced from it) and updates rho, rho v,
# rho w: 80 B + 24 B of w' + 24 B of R_prev (stages 1, 2), a mean of 120 B.
RHS_RK_BYTES_PER_PT = 400.0 / 3.0
RHS_RK_SPLIT_BYTES_PER_PT = 120.0
# FP64 operations of one shock-capturing interface flux in the kernel's
# formulation (weno_node, weno_flux, weno3/5/7, half_sum), counted from the
# source with a fused multiply-add as two, a reciprocal or square root as
# one, comparisons and absolute values as none; by WENO order 2r-1:
#  - the quantities of a node along the direction (reciprocal of the
#    density, velocities, pressure, sound speed: 15), which every node needs
#    once per direction, so one node's worth per interface: 15;
#  - Roe average of nodes i, i+1 from their quantities (reciprocal
#    densities, tangential velocities, enthalpies, square roots, weighted
#    means) and the eigenvector constants: 47;
#  - per stencil node (2r of them): projection of the state on the left
#    eigenvectors 21, projection of the Euler flux from it
#    (u_n L w + p L(0, 1, 0, 0, u_n)) 15, eigenvalue bounds 2: 38;
#  - per characteristic field (5): Lax-Friedrichs splitting 2 (2r - 1) x 2,
#    two reconstructions (WENO3 17, WENO5 61, WENO7 141 each), the half
#    sum of the two with one reciprocal 7;
#  - back-projection on the right eigenvectors: 26.
# WENO5: 15 + 47 + 6 x 38 + 5 x (20 + 122 + 7) + 26 = 1061.  (The kernel
# converts each stencil node of every interface, 2r per interface: a node's
# quantities are computed by each of the 2r interfaces that reach it.)
WENO_FLOPS_BY_ORDER = {3: 505.0, 5: 1061.0, 7: 1977.0}
# Hash of the source region the count was taken from (weno_source_hash());
# a CPU test fails when that code changes, so the count cannot go stale.
WENO_FLOPS_SOURCE_HASH = "f8fa07d7ae70d98f"
WENO_FLOPS_PER_IFACE = WENO_FLOPS_BY_ORDER[5]


# name -> (problem constructor name, description)
WORKLOADS = {
    "channel": ("channel", "compressible channel 256x128x128, FP64 state, hybrid central/WENO "
                           "(Ducros sensor), bulk forcing, tanh-stretched walls, CFL 0.8"),
    "sbli": ("sbli", "oblique shock on a laminar boundary layer 1024x256x128, FP64 state, hybrid "
                     "central/WENO, Dirichlet inflow, characteristic outflow, adiabatic wall, "
                     "imposed shock, CFL 0.8"),
    "tgv": ("taylor_green", "Taylor-Green vortex 32^3, FP64 state, central only, CFL 0.8"),
    "bl": ("boundary_layer", "spatially developing Mach 2 boundary layer 1024x128x128 "
                             "(30 x 12 x 6 inflow thicknesses), FP64 state, hybrid central/WENO, "
                             "digital-filter inflow turbulence, recovery-temperature wall, "
                             "characteristic outflow and top, CFL 0.8"),
}


def kernel_source_hash():
    """Hash of the kernel source without line comments and blank lines, so
    that the stored counter figures stay tied to the code they measured."""
    h = hashlib.sha256()
    for f in ("cdns_kernels.hip",):
        with open(os.path.join(ROOT, "paper_2004_02276_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def weno_source_hash():
    """Hash of the shock-capturing flux code (from the WENO5 reconstruction
    to the end of weno_flux) without comments and blank lines."""
    path = os.path.join(ROOT, "paper_2004_02276_amd", "csrc", "cdns_kernels.hip")
    with open(path, encoding="utf-8") as fh:
        txt = fh.read()
    a = txt.index("// WENO5-JS reconstruction at i+1/2")
    b = txt.index("// ------------------------------------------------------------------ stage begin")
    h = hashlib.sha256()
    for line in txt[a:b].splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, steps, warmup):
    """HBM bytes per launch from committed rocprofv3 counter runs (one entry,
    or a list of entries for several workloads, per kernel), if they were
    taken on the current kernel source, this workload and this step window
    (the channel's shock-capturing share decays over the run, so the bytes
    per launch depend on which steps are timed); else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    ents = t.get(kernel) or []
    if isinstance(ents, dict):  # one workload
        ents = [ents]
    h = kernel_source_hash()
    for ent in ents:
        if (ent.get("source_hash") == h and ent.get("workload") == workload and
                ent.get("steps") == steps and ent.get("warmup") == warmup):
            return ent.get("hbm_bytes_per_launch")
    return None


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Practical HBM rate on this GPU: a device-to-device copy of nbytes,
    (read + written bytes) / mean time of reps copies, GB/s."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def _oracle_rate(pr, budget_s=10.0, max_steps=30):
    """Oracle steps of the full workload from its seeded initial field for
    about budget_s seconds: (Mpoint-RK-steps/s, steps, seconds)."""
    import oracle
    w = pr.w0
    steps = 0
    t0 = time.perf_counter()
    while True:
        w = oracle.advance(pr, 1, w=w, cfl=pr.cfl)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= max_steps:
            break
    return pr.npts * steps / el / 1e6, steps, el


def cpu_baseline(pr, single_thread=False):
    import oracle
    oracle.build(force=False)
    nthreads = oracle.num_threads()
    rate, steps, el = _oracle_rate(pr)  # about 10 s of the host cores
    out = {"value": rate, "unit": "Mpoint-RK-steps/s", "cores": nthreads, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"{steps} RK3 step(s) of the full {pr.name} workload from the same seeded "
                     f"initial field, {el:.1f} s wall"}
    if single_thread:
        prev = oracle.set_threads(1)
        try:
            r1, s1, e1 = _oracle_rate(pr)
        finally:
            oracle.set_threads(prev)
        out["single_thread"] = {"value": r1, "cores": 1,
                                "sample": f"{s1} RK3 step(s), {e1:.1f} s wall"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp64", "fp32flux"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=list(WORKLOADS), default="channel",
                    help="channel (the headline workload); sbli, tgv, bl (reference figures)")
    ap.add_argument("--central-order", type=int, choices=[2, 4, 6], default=4,
                    help="order of the central flux and viscous terms")
    ap.add_argument("--weno-order", type=int, choices=[3, 5, 7], default=5,
                    help="order of the WENO reconstruction")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (one simulation "
              "per GPU; see DESIGN.md for how the step would shard). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import problems as P
    from paper_2004_02276_amd import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    # one device-to-device copy of known size (256 MiB read + 256 MiB written):
    # reference dispatch for scaling the HBM byte counters of a profiled run
    src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    copy_gbs = copy_bandwidth(torch)
    pr = getattr(P, WORKLOADS[args.workload][0])()
    pr = dataclasses.replace(pr, central_order=args.central_order, weno_order=args.weno_order)
    # counter-based traffic figures were taken with the default scheme
    default_scheme = (args.central_order, args.weno_order) == (4, 5)
    precision = 0 if args.precision == "fp64" else 1
    s = Solver(pr, precision=precision)
    cfl = pr.cfl
    print(f"# workload {pr.name} {pr.npts} points, warmup {args.warmup}", file=sys.stderr,
          flush=True)
    s.advance(args.warmup, cfl=cfl)
    torch.cuda.synchronize()
    with torch.cuda.stream(s.stream):
        start_state = s.state.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(args.steps, cfl=cfl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = s.diagnostics()
    el = t1 - t0
    ms_per_step = el * 1e3 / args.steps
    value = pr.npts * args.steps / el / 1e6
    print(f"# timed {args.steps} steps in {el:.3f} s, weno fraction {d['weno_frac']}",
          file=sys.stderr, flush=True)

    # per-kernel durations with HIP events over the same steps: the state is
    # rewound to the start of the timed region and the steps are replayed
    # kernel by kernel with an event pair around every launch
    s.set_state(start_state)
    torch.cuda.synchronize()
    ph, n_iface_total = s.time_phases(args.steps, cfl=cfl, with_interfaces=True)
    per_step = {k: v[0] * v[1] / args.steps for k, v in ph.items()}
    dom = max(per_step, key=per_step.get)
    mean_ms = ph[dom][0]
    if dom == "weno":
        n_iface = n_iface_total / max(ph["weno"][1], 1)
        fl_if = WENO_FLOPS_BY_ORDER[args.weno_order]
        flops = fl_if * n_iface
        achieved = flops / (mean_ms * 1e-3) / 1e12
        roof = {"kernel": "k_weno", "bound": "alu", "achieved": achieved,
                "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_TFLOPS,
                "traffic": load_traffic("k_weno", args.workload, args.steps, args.warmup)
                           if default_scheme else None,
                "algorithmic_per_launch": f"{fl_if:.0f} flop x {n_iface:.0f} "
                                          f"interfaces (mean over the timed launches)"}
    else:
        # the default 64x4 tiling (the one used here) does the stage update
        # inside the flux kernel: whole without forcing (no update
        # launches), the part without the force otherwise
        bpp = RHS_RK_SPLIT_BYTES_PER_PT if pr.forcing else RHS_RK_BYTES_PER_PT
        nbytes = bpp * pr.npts
        achieved = nbytes / (ph["rhs"][0] * 1e-3) / 1e9
        roof = {"kernel": "k_rhs", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": load_traffic("k_rhs", args.workload, args.steps, args.warmup)
                           if default_scheme else None,
                "algorithmic_per_launch": f"{bpp:.1f} B x {pr.npts} points (RK update included)"}
    roof["mean_launch_ms"] = mean_ms
    scheme = ("" if (args.central_order, args.weno_order) == (4, 5) else
              f"; central order {args.central_order}, WENO order {args.weno_order}")
    step_bytes = STEP_BYTES_PER_PT_FORCED if pr.forcing else STEP_BYTES_PER_PT
    hbm_frac_step = value * 1e6 * step_bytes / (HBM_PEAK_GBS * 1e9)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Mpoint-RK-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][1] + scheme,
                   "points": pr.npts, "parallelism": "single GPU"},
        "hbm_frac_step_algorithmic": hbm_frac_step,
        "phase_ms_per_step": per_step,
        "weno_frac_last_stage": d["weno_frac"],
        "weno_interfaces_per_step": n_iface_total / args.steps,
        "roofline": roof,
        "hbm_copy_GBps": copy_gbs,
    }
    s.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr, single_thread=(args.workload == "tgv"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
