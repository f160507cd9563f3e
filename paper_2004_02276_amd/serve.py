"""Continuous-batching serving of many independent simulations on one GPU.

`Batch` wraps the batched runner of libcdns.so: every attached instance is
advanced by each batch step, one persistent kernel per phase covering all
instances, the whole step replayed from one HIP graph.  `Server` runs a
trace of requests: requests are admitted in arrival order as slots and
the HBM budget allow (state + workspace of the instance), join the batch,
are advanced together with whatever else is resident, and retire after
their step count -- freeing memory and a slot for the next.  Between two
host checks the batch replays up to `max_chunk` steps: as many as no
resident request overruns its step count and the next arrival is not
expected to be kept waiting (from the measured step time), so the GPU does
not idle while the host does its bookkeeping after every step.
Per-request step latencies are the wall-clock time of each replay divided
evenly over its steps.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import _binding as B
from .solver import Solver


class Batch:
    def __init__(self, max_slots: int = 64, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.lib = B.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        wsb = self.lib.cdns_batch_workspace_bytes(int(max_slots))
        if wsb == 0:
            raise B.CdnsError(B.CDNS_EINVAL, "max_slots out of range")
        self._ws = torch.empty(wsb + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.h = ctypes.c_void_p()
        B.check(self.lib, None,
                self.lib.cdns_batch_create(int(max_slots), ptr, wsb,
                                           ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(self.h)), "cdns_batch_create")
        self.max_slots = max_slots

    def attach(self, solver: Solver, cfl: Optional[float] = None, dt_fixed: float = 0.0) -> int:
        slot = ctypes.c_int32(-1)
        B.check(self.lib, None, self.lib.cdns_batch_attach(self.h, solver.ctx, ctypes.byref(slot)),
                "cdns_batch_attach")
        cfl = solver.pr.cfl if cfl is None else cfl
        B.check(self.lib, None,
                self.lib.cdns_batch_set_step(self.h, slot.value, float(cfl), float(dt_fixed)),
                "cdns_batch_set_step")
        return slot.value

    def detach(self, slot: int) -> None:
        B.check(self.lib, None, self.lib.cdns_batch_detach(self.h, int(slot)), "cdns_batch_detach")

    def step(self, n: int = 1) -> None:
        B.check(self.lib, None, self.lib.cdns_batch_step(self.h, int(n)), "cdns_batch_step")

    def close(self) -> None:
        if self.h:
            self.stream.synchronize()
            self.lib.cdns_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint_bytes(problem, precision: int = 0) -> int:
    """Device bytes one instance holds while resident: state + workspace."""
    lib = B.load()
    ye = np.ascontiguousarray(problem.y_eta, dtype=np.float64)
    yee = np.ascontiguousarray(problem.y_etaeta, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    g = B.Grid(problem.nx, problem.ny, problem.nz, problem.lx, problem.lz,
               ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    return int(lib.cdns_workspace_bytes(ctypes.byref(g), precision)) + 40 * problem.npts + 512


@dataclasses.dataclass
class RequestResult:
    rid: int
    npts: int
    arrival: float
    admitted: float = -1.0
    finished: float = -1.0
    steps: int = 0
    step_latencies: List[float] = dataclasses.field(default_factory=list)
    status: str = "pending"
    state: Optional[np.ndarray] = None


class Server:
    """Admission by HBM budget + continuous batching of resident instances.

    make_problem(spec) builds the request's Problem (grid, parameters and
    initial field); specs need .rid, .arrival (s) and .nsteps."""

    def __init__(self, make_problem, hbm_budget_bytes: int, max_slots: int = 64,
                 tiling=(64, 4), kz_for=None, keep_states: bool = False, device: str = "cuda:0",
                 max_chunk: int = 8):
        import torch
        self.torch = torch
        self.max_chunk = max(1, int(max_chunk))
        self.make_problem = make_problem
        self.budget = int(hbm_budget_bytes)
        self.max_slots = max_slots
        self.tiling = tiling
        self.kz_for = kz_for or (lambda pr: 16)
        self.keep_states = keep_states
        self.device = device

    def _admit(self, spec, pr, now, batch, resident, used):
        """Make the instance resident; (used bytes, False) if the batched
        kernels do not run its configuration (digital-filter inflow or
        scheme orders other than 4/5)."""
        s = Solver(pr, device=self.device, tiling=(self.tiling[0], self.tiling[1], self.kz_for(pr)))
        try:
            slot = batch.attach(s)
        except B.CdnsError as err:
            s.close()
            if err.status != B.CDNS_EUNSUP:
                raise
            return used, False
        resident[spec.rid] = (spec, s, slot)
        return used + footprint_bytes(pr), True

    def run(self, specs, mode: str = "batch", prebuilt: Optional[Dict] = None) -> Dict:
        """Serve the trace.  mode 'batch' (continuous batching) or 'serial'
        (FIFO, one request at a time through Solver.advance)."""
        torch = self.torch
        specs = sorted(specs, key=lambda s: (s.arrival, s.rid))
        problems = prebuilt if prebuilt is not None else {s.rid: self.make_problem(s) for s in specs}
        results = {s.rid: RequestResult(s.rid, problems[s.rid].npts, s.arrival) for s in specs}
        pending = list(specs)
        queue: List = []
        resident: Dict = {}
        used = 0
        batch = Batch(self.max_slots, device=self.device) if mode == "batch" else None
        total_pts = 0
        t0 = time.perf_counter()
        peak_used = 0
        waited = set()      # requests that found the budget full on arrival
        t_step = None       # measured wall time of one batch step (latest)
        while pending or queue or resident:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            if mode == "batch":
                # admit in arrival order while memory and slots allow
                while queue and len(resident) < self.max_slots:
                    spec = queue[0]
                    need = footprint_bytes(problems[spec.rid])
                    if need > self.budget:
                        queue.pop(0)
                        results[spec.rid].status = "rejected: larger than the budget"
                        continue
                    if used + need > self.budget:
                        waited.update(q.rid for q in queue)
                        break
                    queue.pop(0)
                    used, ok = self._admit(spec, problems[spec.rid], now, batch, resident, used)
                    if not ok:
                        results[spec.rid].status = "rejected: configuration not batchable"
                        continue
                    peak_used = max(peak_used, used)
                    results[spec.rid].admitted = time.perf_counter() - t0
                if not resident:
                    if pending:
                        time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                    continue
                # steps until the first resident finishes, and until the next
                # arrival (at the measured step time)
                k = min(self.max_chunk,
                        min(sp.nsteps - results[rid].steps for rid, (sp, _, _) in resident.items()))
                if pending and t_step:
                    ahead = pending[0].arrival - (time.perf_counter() - t0)
                    k = min(k, max(1, int(ahead / t_step)))
                t_a = time.perf_counter()
                batch.step(k)
                torch.cuda.synchronize()
                tnow = time.perf_counter()
                t_step = (tnow - t_a) / k
                finished = []
                for rid, (spec, s, slot) in resident.items():
                    r = results[rid]
                    r.step_latencies.extend([t_step] * k)
                    r.steps += k
                    total_pts += r.npts * k
                    if r.steps >= spec.nsteps:
                        finished.append(rid)
                for rid in finished:
                    spec, s, slot = resident.pop(rid)
                    batch.detach(slot)
                    self._retire(s, results[rid], t0)
                    used -= footprint_bytes(problems[rid])
            else:
                if not queue:
                    if pending:
                        time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                    continue
                spec = queue.pop(0)
                pr = problems[spec.rid]
                r = results[spec.rid]
                s = Solver(pr, device=self.device,
                           tiling=(self.tiling[0], self.tiling[1], self.kz_for(pr)))
                r.admitted = time.perf_counter() - t0
                last = time.perf_counter()
                for _ in range(spec.nsteps):
                    s.advance(1, cfl=pr.cfl)
                    torch.cuda.synchronize()
                    tnow = time.perf_counter()
                    r.step_latencies.append(tnow - last)
                    last = tnow
                    r.steps += 1
                total_pts += r.npts * spec.nsteps
                self._retire(s, r, t0)
        makespan = time.perf_counter() - t0
        if batch is not None:
            batch.close()
        lat = np.concatenate([np.array(r.step_latencies) for r in results.values()
                              if r.step_latencies]) if results else np.zeros(0)
        return {
            "mode": mode,
            "makespan_s": makespan,
            "throughput_mpts": total_pts / makespan / 1e6,
            "p50_step_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_step_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in results.values()
                                           if r.admitted >= 0])),
            "mean_e2e_s": float(np.mean([r.finished - r.arrival for r in results.values()
                                         if r.finished >= 0])),
            "peak_resident_bytes": peak_used,
            "budget_bytes": self.budget,
            "waited_for_memory": len(waited),
            "max_chunk": self.max_chunk if mode == "batch" else 1,
            "completed": sum(r.status == "ok" for r in results.values()),
            "failed": sum(r.status.startswith("failed") for r in results.values()),
            "rejected": sum(r.status.startswith("rejected") for r in results.values()),
            "results": results,
        }

    def _retire(self, s: Solver, r: RequestResult, t0: float) -> None:
        d = s.diagnostics(raise_on_error=False)
        r.status = "ok" if d["rc"] == 0 else f"failed: status {d['status']}"
        if self.keep_states:
            r.state = s.get_state()
        r.finished = time.perf_counter() - t0
        s.close()
