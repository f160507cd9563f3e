#!/usr/bin/env python3
"""Serving benchmark: a Poisson stream of independent simulations.

64 requests (mean 4 arrivals/s, seeded), each a periodic decaying
turbulence box carried by a uniform stream or a channel, cubic grid N^3
with N uniform in [32, 192], Mach in [0.1, 3], Re in [500, 5000], 200 RK
steps, FP64 state.  Runs the trace twice on one GPU: continuous batching
(admission by an HBM budget, one persistent kernel per phase for all
resident instances, graph-replayed batch steps) and serially (FIFO, one
request at a time), and prints one JSON line with throughput and p50/p99
step latency of both.

Options scale the trace down for quick checks (--requests, --nmax,
--steps) or remove arrivals (--burst).
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
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--nmin", type=int, default=32)
    ap.add_argument("--nmax", type=int, default=192)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="HBM budget for resident instances (0: 80%% of free memory)")
    ap.add_argument("--burst", action="store_true")
    ap.add_argument("--skip-serial", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip tuning kz per size class (use the cached or heuristic value)")
    ap.add_argument("--batch-kz", type=int, default=32,
                    help="z planes per fused-kernel block in batch mode (0: the per-instance "
                         "tuned or heuristic value, as in serial mode)")
    ap.add_argument("--max-chunk", type=int, default=8,
                    help="batch steps replayed between host checks at most")
    args = ap.parse_args()

    import torch

    import problems as P
    from paper_2004_02276_amd import autotune
    from paper_2004_02276_amd.serve import Server

    specs = P.serving_trace(args.requests, args.rate, args.nmin, args.nmax, nsteps=args.steps,
                            burst=args.burst)
    t0 = time.perf_counter()
    prebuilt = {s.rid: P.request_problem(s) for s in specs}
    print(f"# built {len(specs)} request inputs in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * 1e9) if args.budget_gb > 0 else int(0.8 * free)
    tile = (64, 4)  # instances of one batch share the tile shape; kz is per instance
    tuned = {}
    if not args.no_tune:
        # one representative request per size class, tuned before serving
        t0 = time.perf_counter()
        for sp in specs:
            cls = autotune.size_class(prebuilt[sp.rid])
            if cls not in tuned:
                res = autotune.tune(prebuilt[sp.rid], 0, steps=2, fixed_tile=tile, save=False)
                tuned[cls] = res["kz"]
        print(f"# tuned kz for {len(tuned)} size classes in {time.perf_counter() - t0:.1f} s: "
              f"{tuned}", file=sys.stderr, flush=True)
    kz_for = lambda pr: tuned.get(autotune.size_class(pr),
                                  autotune.lookup(pr, 0, fixed_tile=tile)[2])
    # the per-class values are tuned on one instance alone, where small
    # instances need shallow z chunks to fill the GPU; in a batch the
    # residents fill it together, and deep chunks re-read fewer halo planes
    batch_kz_for = (lambda pr: min(args.batch_kz, pr.nz)) if args.batch_kz > 0 else kz_for
    out = {"metric": "batched serving throughput and p50/p99 step latency",
           "requests": len(specs), "rate_per_s": args.rate, "steps": args.steps,
           "grid_range": [args.nmin, args.nmax], "budget_gb": budget / 1e9,
           "total_mpoint_steps": sum(s.n ** 3 * s.nsteps for s in specs) / 1e6,
           "tuned_kz": tuned, "batch_kz": args.batch_kz, "max_chunk": args.max_chunk}
    for mode in (["batch"] if args.skip_serial else ["batch", "serial"]):
        srv = Server(P.request_problem, budget, max_slots=64, tiling=tile,
                     kz_for=batch_kz_for if mode == "batch" else kz_for, max_chunk=args.max_chunk)
        rep = srv.run(specs, mode=mode, prebuilt=prebuilt)
        rep.pop("results")
        out[mode] = rep
        print(f"# {mode}: {json.dumps(rep)}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
    if "serial" in out:
        out["throughput_speedup_vs_serial"] = (out["batch"]["throughput_mpts"]
                                              / out["serial"]["throughput_mpts"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
