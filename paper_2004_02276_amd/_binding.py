"""ctypes binding of libcdns.so (argument marshalling only).

Every numerical step runs inside the HIP library; PyTorch only allocates
device memory and supplies the stream.  If the library is missing the import
of this module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdns.so")

CDNS_OK, CDNS_EINVAL, CDNS_ENOMEM, CDNS_EHIP, CDNS_ESTATE, CDNS_EUNSUP, CDNS_EBUSY = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "EUNSUP",
                -6: "EBUSY"}
CDNS_FP64, CDNS_FP32_FLUX = 0, 1
PHASES = ["dt", "ghosts", "sensor", "iflags", "weno", "rhs", "force", "rk"]
NSTAT = 16  # running-statistics products (CDNS_NSTAT)
MEAN_NAMES = ["rho", "u_favre", "v_favre", "w_favre", "R11", "R22", "R33", "R12", "u", "u_rms",
              "T", "T_favre", "T_rms", "p", "p_rms", "rho_rms"]  # CDNS_MN_* order
NDIAG_DEV = 10  # slots of cdns_diagnostics_noalloc's output (CDNS_NDIAG_DEV)
DIAG_DEV_NAMES = ["mass", "mom_x", "mom_y", "mom_z", "energy", "kinetic", "rho_min", "p_min",
                  "mach_max", "nonfinite"]
NOALLOC_MAX_POINTS = 33554432  # CDNS_NOALLOC_MAX_POINTS

EXPORTED = [
    "cdns_version", "cdns_workspace_bytes", "cdns_create", "cdns_set_bc", "cdns_set_tiling",
    "cdns_set_scheme", "cdns_set_state", "cdns_get_state", "cdns_export_flags",
    "cdns_import_flags", "cdns_poison_workspace",
    "cdns_rhs", "cdns_rk_step", "cdns_advance_n", "cdns_diagnostics",
    "cdns_diagnostics_noalloc", "cdns_export_sensor",
    "cdns_export_iface_flux", "cdns_time_phases", "cdns_stats_accumulate", "cdns_stats_export",
    "cdns_stats_reset", "cdns_stats_means",
    "cdns_last_error", "cdns_destroy", "cdns_batch_create", "cdns_batch_workspace_bytes",
    "cdns_batch_attach", "cdns_batch_detach", "cdns_batch_set_step", "cdns_batch_step",
    "cdns_batch_destroy",
]


class CdnsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("lz", ctypes.c_double),
                ("y_eta", ctypes.POINTER(ctypes.c_double)),
                ("y_etaeta", ctypes.POINTER(ctypes.c_double))]


class Phys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("R_gas", ctypes.c_double),
                ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("S_suth", ctypes.c_double), ("viscous", ctypes.c_int32),
                ("sensor_mode", ctypes.c_int32), ("theta_star", ctypes.c_double),
                ("sensor_eps", ctypes.c_double), ("forcing", ctypes.c_int32)]


class Diag(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("time", ctypes.c_double), ("mass", ctypes.c_double),
                ("mom", ctypes.c_double * 3), ("energy", ctypes.c_double),
                ("kinetic", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("p_min", ctypes.c_double), ("mach_max", ctypes.c_double),
                ("forcing_f", ctypes.c_double), ("weno_frac", ctypes.c_double * 3),
                ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
                ("status", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libcdns.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2004_02276_amd/build.py "
                          "(the HIP library is required; there is no CPU path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.c_void_p  # device pointers are passed as integers
    i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.cdns_version.restype = ctypes.c_char_p
    lib.cdns_workspace_bytes.argtypes = [ctypes.POINTER(Grid), i32]
    lib.cdns_workspace_bytes.restype = sz
    lib.cdns_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Phys), i32, dp, dp, sz, vp,
                                ctypes.POINTER(vp)]
    lib.cdns_create.restype = i32
    lib.cdns_set_bc.argtypes = [vp, i32, i32, ctypes.POINTER(f64), i64]
    lib.cdns_set_bc.restype = i32
    lib.cdns_poison_workspace.argtypes = [vp]
    lib.cdns_poison_workspace.restype = i32
    lib.cdns_set_tiling.argtypes = [vp, i32, i32, i32]
    lib.cdns_set_tiling.restype = i32
    lib.cdns_set_scheme.argtypes = [vp, i32, i32]
    lib.cdns_set_scheme.restype = i32
    lib.cdns_set_state.argtypes = [vp, vp, i32]
    lib.cdns_set_state.restype = i32
    lib.cdns_get_state.argtypes = [vp, vp, i32]
    lib.cdns_get_state.restype = i32
    lib.cdns_export_flags.argtypes = [vp, dp]
    lib.cdns_export_flags.restype = i32
    lib.cdns_import_flags.argtypes = [vp, dp]
    lib.cdns_import_flags.restype = i32
    lib.cdns_rhs.argtypes = [vp, dp, dp]
    lib.cdns_rhs.restype = i32
    lib.cdns_rk_step.argtypes = [vp, f64, f64]
    lib.cdns_rk_step.restype = i32
    lib.cdns_advance_n.argtypes = [vp, i32, f64, f64]
    lib.cdns_advance_n.restype = i32
    lib.cdns_diagnostics.argtypes = [vp, ctypes.POINTER(Diag)]
    lib.cdns_diagnostics.restype = i32
    lib.cdns_diagnostics_noalloc.argtypes = [vp, dp, dp]
    lib.cdns_diagnostics_noalloc.restype = i32
    lib.cdns_export_sensor.argtypes = [vp, dp, dp, dp]
    lib.cdns_export_sensor.restype = i32
    lib.cdns_export_iface_flux.argtypes = [vp, i32, dp]
    lib.cdns_export_iface_flux.restype = i32
    lib.cdns_time_phases.argtypes = [vp, i32, f64, f64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.cdns_time_phases.restype = i32
    lib.cdns_stats_accumulate.argtypes = [vp]
    lib.cdns_stats_accumulate.restype = i32
    lib.cdns_stats_export.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]
    lib.cdns_stats_export.restype = i32
    lib.cdns_stats_reset.argtypes = [vp]
    lib.cdns_stats_reset.restype = i32
    lib.cdns_stats_means.argtypes = [vp, i32, dp]
    lib.cdns_stats_means.restype = i32
    lib.cdns_last_error.argtypes = [vp]
    lib.cdns_last_error.restype = ctypes.c_char_p
    lib.cdns_destroy.argtypes = [vp]
    lib.cdns_destroy.restype = i32
    lib.cdns_batch_workspace_bytes.argtypes = [i32]
    lib.cdns_batch_workspace_bytes.restype = sz
    lib.cdns_batch_create.argtypes = [i32, dp, sz, vp, ctypes.POINTER(vp)]
    lib.cdns_batch_create.restype = i32
    lib.cdns_batch_attach.argtypes = [vp, vp, ctypes.POINTER(i32)]
    lib.cdns_batch_attach.restype = i32
    lib.cdns_batch_detach.argtypes = [vp, i32]
    lib.cdns_batch_detach.restype = i32
    lib.cdns_batch_set_step.argtypes = [vp, i32, f64, f64]
    lib.cdns_batch_set_step.restype = i32
    lib.cdns_batch_step.argtypes = [vp, i32]
    lib.cdns_batch_step.restype = i32
    lib.cdns_batch_destroy.argtypes = [vp]
    lib.cdns_batch_destroy.restype = i32
    _lib = lib
    return lib


def check(lib, ctx, status: int, what: str):
    if status != CDNS_OK:
        msg = lib.cdns_last_error(ctx).decode() if ctx else ""
        raise CdnsError(status, f"{what}: {msg}")
