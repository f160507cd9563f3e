"""Python front end of the HIP solver: one instance on one GPU.

`Solver` owns torch tensors for the state and the workspace and forwards
every operation to libcdns.so; it performs no arithmetic of its own.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

import numpy as np

from . import _binding as B


class Solver:
    """A resident instance of the right-hand side / RK3 stepper.

    `problem` is any object with the fields of `problems.Problem`
    (grid sizes, lengths, metric arrays, physical parameters, boundary
    conditions and an initial state w0 of shape (5, nz, ny, nx))."""

    def __init__(self, problem, precision: int = B.CDNS_FP64, device: str = "cuda:0",
                 tiling=None, stream=None):
        import torch

        self.torch = torch
        self.lib = B.load()
        self.pr = problem
        self.device = torch.device(device)
        self.precision = int(precision)
        nx, ny, nz = problem.nx, problem.ny, problem.nz
        self._ye = np.ascontiguousarray(problem.y_eta, dtype=np.float64)
        self._yee = np.ascontiguousarray(problem.y_etaeta, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        self.grid = B.Grid(nx, ny, nz, problem.lx, problem.lz,
                           self._ye.ctypes.data_as(dp), self._yee.ctypes.data_as(dp))
        self.phys = B.Phys(problem.gamma, problem.Pr, problem.R_gas, problem.mu_ref,
                           problem.T_ref, problem.S_suth, int(bool(problem.viscous)),
                           int(problem.sensor_mode), problem.theta_star, problem.sensor_eps,
                           int(bool(problem.forcing)))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.state = torch.empty((5, nz, ny, nx), dtype=torch.float64, device=self.device)
        wsb = self.lib.cdns_workspace_bytes(ctypes.byref(self.grid), self.precision)
        if wsb == 0:
            raise B.CdnsError(B.CDNS_EINVAL, "invalid grid")
        self._ws = torch.empty(wsb + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = ctypes.c_void_p()
        st = self.lib.cdns_create(ctypes.byref(self.grid), ctypes.byref(self.phys),
                                  self.precision, self.state.data_ptr(), self._ws_ptr, wsb,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx))
        B.check(self.lib, None, st, "cdns_create")
        for face, (kind, params) in enumerate(problem.bcs):
            arr = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
            ptr = arr.ctypes.data_as(dp) if arr.size else None
            B.check(self.lib, self.ctx,
                    self.lib.cdns_set_bc(self.ctx, face, int(kind), ptr, arr.size), "cdns_set_bc")
        co = int(getattr(problem, "central_order", 4))
        wo = int(getattr(problem, "weno_order", 5))
        if (co, wo) != (4, 5):
            self.set_scheme(co, wo)
        if tiling is not None:
            self.set_tiling(*tiling)
        if problem.w0 is not None:
            self.set_state(problem.w0)

    # ------------------------------------------------------------ state
    def set_state(self, w) -> None:
        """Copy a state (host numpy array or device tensor) into the solver."""
        t = self.torch
        if isinstance(w, np.ndarray):
            h = np.ascontiguousarray(w, dtype=np.float64)
            assert h.size == self.state.numel()
            B.check(self.lib, self.ctx, self.lib.cdns_set_state(self.ctx, h.ctypes.data, 1),
                    "cdns_set_state")
            return
        d = w.to(self.device, dtype=t.float64).contiguous()
        assert d.numel() == self.state.numel()
        B.check(self.lib, self.ctx, self.lib.cdns_set_state(self.ctx, d.data_ptr(), 0),
                "cdns_set_state")
        self.stream.synchronize()  # keeps d alive until the copy is done

    def get_state(self) -> np.ndarray:
        out = np.empty(tuple(self.state.shape), dtype=np.float64)
        B.check(self.lib, self.ctx, self.lib.cdns_get_state(self.ctx, out.ctypes.data, 1),
                "cdns_get_state")
        return out

    def export_flags(self):
        """Node flags of the last right-hand side (device uint8 tensor)."""
        t = self.torch
        out = t.empty((self.pr.nz, self.pr.ny, self.pr.nx), dtype=t.uint8, device=self.device)
        B.check(self.lib, self.ctx, self.lib.cdns_export_flags(self.ctx, out.data_ptr()),
                "cdns_export_flags")
        return out

    def import_flags(self, flags) -> None:
        """Node flags to use in the next right-hand side instead of the sensor."""
        t = self.torch
        if isinstance(flags, np.ndarray):
            flags = t.from_numpy(np.ascontiguousarray(flags, dtype=np.uint8))
        d = flags.to(self.device, dtype=t.uint8).contiguous()
        assert d.numel() == self.state.numel() // 5
        B.check(self.lib, self.ctx, self.lib.cdns_import_flags(self.ctx, d.data_ptr()),
                "cdns_import_flags")
        self.stream.synchronize()

    def poison_workspace(self) -> None:
        """Fill the work regions of the workspace with NaN (debugging: reads
        of memory no kernel has written then show up in the results)."""
        B.check(self.lib, self.ctx, self.lib.cdns_poison_workspace(self.ctx),
                "cdns_poison_workspace")

    # ------------------------------------------------------------ operations
    def set_tiling(self, tile_x: int, tile_y: int, kz: int) -> None:
        B.check(self.lib, self.ctx, self.lib.cdns_set_tiling(self.ctx, tile_x, tile_y, kz),
                "cdns_set_tiling")

    def set_scheme(self, central_order: int, weno_order: int) -> None:
        """Central/viscous order (2, 4, 6) and WENO order (3, 5, 7)."""
        B.check(self.lib, self.ctx,
                self.lib.cdns_set_scheme(self.ctx, int(central_order), int(weno_order)),
                "cdns_set_scheme")

    def rhs(self, w=None, out=None):
        t = self.torch
        if w is None:
            w = self.state
        elif isinstance(w, np.ndarray):
            w = t.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).to(self.device)
        w = w.contiguous()
        if out is None:
            out = t.empty_like(w)
        B.check(self.lib, self.ctx, self.lib.cdns_rhs(self.ctx, w.data_ptr(), out.data_ptr()),
                "cdns_rhs")
        return out

    def rk_step(self, cfl: Optional[float] = None, dt_fixed: float = 0.0) -> None:
        cfl = self.pr.cfl if cfl is None else cfl
        B.check(self.lib, self.ctx, self.lib.cdns_rk_step(self.ctx, float(cfl), float(dt_fixed)),
                "cdns_rk_step")

    def advance(self, n: int, cfl: Optional[float] = None, dt_fixed: float = 0.0) -> None:
        cfl = self.pr.cfl if cfl is None else cfl
        B.check(self.lib, self.ctx,
                self.lib.cdns_advance_n(self.ctx, int(n), float(cfl), float(dt_fixed)),
                "cdns_advance_n")

    def diagnostics(self, raise_on_error: bool = True) -> Dict:
        d = B.Diag()
        st = self.lib.cdns_diagnostics(self.ctx, ctypes.byref(d))
        if raise_on_error:
            B.check(self.lib, self.ctx, st, "cdns_diagnostics")
        return {"dt": d.dt, "time": d.time, "mass": d.mass, "mom": list(d.mom),
                "energy": d.energy, "kinetic": d.kinetic, "rho_min": d.rho_min,
                "p_min": d.p_min, "mach_max": d.mach_max, "forcing_f": d.forcing_f,
                "weno_frac": list(d.weno_frac), "step": d.step, "nonfinite": d.nonfinite,
                "status": d.status, "rc": st}

    def diagnostics_noalloc(self, w=None, out=None):
        """Volume integrals and extrema (B.DIAG_DEV_NAMES) of the state, or of
        the device tensor w, written on the device into out (a float64 tensor
        of B.NDIAG_DEV values, created if None) without synchronising."""
        t = self.torch
        if out is None:
            out = t.empty(B.NDIAG_DEV, dtype=t.float64, device=self.device)
        assert out.dtype == t.float64 and out.numel() >= B.NDIAG_DEV and out.is_contiguous()
        if w is not None:
            assert w.dtype == t.float64 and w.numel() == self.state.numel() and w.is_contiguous()
        wp = w.data_ptr() if w is not None else None
        B.check(self.lib, self.ctx,
                self.lib.cdns_diagnostics_noalloc(self.ctx, wp, out.data_ptr()),
                "cdns_diagnostics_noalloc")
        return out

    def export_sensor(self):
        t = self.torch
        shp = (self.pr.nz, self.pr.ny, self.pr.nx)
        theta = t.empty(shp, dtype=t.float64, device=self.device)
        nfl = t.empty(shp, dtype=t.uint8, device=self.device)
        ifl = t.empty(shp, dtype=t.uint8, device=self.device)
        B.check(self.lib, self.ctx,
                self.lib.cdns_export_sensor(self.ctx, theta.data_ptr(), nfl.data_ptr(),
                                            ifl.data_ptr()), "cdns_export_sensor")
        return theta, nfl, ifl

    # ------------------------------------------------------------ statistics
    def stats_accumulate(self) -> None:
        """Add the spanwise sums of the current state's statistics products
        to the running accumulator (asynchronous)."""
        B.check(self.lib, self.ctx, self.lib.cdns_stats_accumulate(self.ctx),
                "cdns_stats_accumulate")

    def stats_reset(self) -> None:
        B.check(self.lib, self.ctx, self.lib.cdns_stats_reset(self.ctx), "cdns_stats_reset")

    def stats_raw(self):
        """(sums [16][ny][nx] over z and samples, number of samples)."""
        out = np.zeros((B.NSTAT, self.pr.ny, self.pr.nx))
        n = ctypes.c_int64(0)
        B.check(self.lib, self.ctx,
                self.lib.cdns_stats_export(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           ctypes.byref(n)), "cdns_stats_export")
        return out, int(n.value)

    def stats(self, average_x: bool = False) -> Dict:
        """Mean fields from the running statistics (computed by the library,
        cdns_stats_means): spanwise (and, with average_x, streamwise)
        Reynolds and Favre means, Favre stresses R11, R22, R33, R12, rms of
        u, T, p and rho; arrays over (y, x), or over y with average_x."""
        t = self.torch
        shp = (B.NSTAT, self.pr.ny) if average_x else (B.NSTAT, self.pr.ny, self.pr.nx)
        out = t.empty(shp, dtype=t.float64, device=self.device)
        B.check(self.lib, self.ctx,
                self.lib.cdns_stats_means(self.ctx, int(bool(average_x)), out.data_ptr()),
                "cdns_stats_means")
        self.stream.synchronize()
        host = out.cpu().numpy()
        res = {name: host[q] for q, name in enumerate(B.MEAN_NAMES)}
        res["samples"] = self.stats_raw()[1]
        return res

    def export_iface_flux(self, d: int):
        t = self.torch
        out = t.empty((5, self.pr.nz, self.pr.ny, self.pr.nx), dtype=t.float64, device=self.device)
        B.check(self.lib, self.ctx, self.lib.cdns_export_iface_flux(self.ctx, d, out.data_ptr()),
                "cdns_export_iface_flux")
        return out

    def time_phases(self, nsteps: int, cfl: Optional[float] = None, dt_fixed: float = 0.0,
                    with_interfaces: bool = False):
        """Mean duration (ms) and count of one launch of each kernel phase over
        nsteps eagerly launched steps, timed with HIP events on the stream.
        With with_interfaces, also the total number of shock-capturing
        interfaces processed by the timed WENO launches: (phases, total)."""
        cfl = self.pr.cfl if cfl is None else cfl
        n = len(B.PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        nif = ctypes.c_int64(0)
        B.check(self.lib, self.ctx,
                self.lib.cdns_time_phases(self.ctx, int(nsteps), float(cfl), float(dt_fixed), ms,
                                          cnt, ctypes.byref(nif)), "cdns_time_phases")
        ph = {B.PHASES[i]: (ms[i], cnt[i]) for i in range(n)}
        return (ph, int(nif.value)) if with_interfaces else ph

    def close(self) -> None:
        if self.ctx:
            self.stream.synchronize()
            self.lib.cdns_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
