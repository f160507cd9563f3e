"""CPU checks of the C ABI: the HIP library loads and exports every function
declared in include/cdns.h; host-only entry points behave without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "cdns.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cdns_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["cdns_create", "cdns_set_bc", "cdns_rhs", "cdns_rk_step", "cdns_advance_n",
                 "cdns_diagnostics", "cdns_destroy", "cdns_batch_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2004_02276_amd import _binding as B
    lib = B.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(B.EXPORTED) >= set(declared_functions())


def test_workspace_size_is_host_only_and_validates():
    from paper_2004_02276_amd import _binding as B
    lib = B.load()
    ye = np.full(16, 2.0)
    yee = np.zeros(16)
    dp = ctypes.POINTER(ctypes.c_double)
    g = B.Grid(32, 16, 8, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    n = lib.cdns_workspace_bytes(ctypes.byref(g), 0)
    N = 32 * 16 * 8
    assert n > 5 * N * 8 * 4  # stage states and residual registers at least
    assert n % 256 == 0
    g_bad = B.Grid(2, 16, 8, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    assert lib.cdns_workspace_bytes(ctypes.byref(g_bad), 0) == 0
    assert lib.cdns_workspace_bytes(ctypes.byref(g), 7) == 0


def test_workspace_size_at_the_largest_grid():
    # node indices are 32-bit inside the kernels: a grid of 2^31 nodes or
    # more is rejected, one just below is sized (its workspace, 100 GB and
    # more, is then a matter for the device's memory)
    from paper_2004_02276_amd import _binding as B
    lib = B.load()
    dp = ctypes.POINTER(ctypes.c_double)
    ye = np.full(1024, 2.0)
    yee = np.zeros(1024)
    g_max = B.Grid(2047, 1024, 1024, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    n = lib.cdns_workspace_bytes(ctypes.byref(g_max), 0)
    N = 2047 * 1024 * 1024
    assert N < 2 ** 31 and n > 5 * N * 8 * 4 and n % 256 == 0
    g_over = B.Grid(2048, 1024, 1024, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    assert lib.cdns_workspace_bytes(ctypes.byref(g_over), 0) == 0


def test_create_rejects_bad_arguments_before_touching_the_device():
    from paper_2004_02276_amd import _binding as B
    lib = B.load()
    ye = np.full(16, 2.0)
    yee = np.zeros(16)
    dp = ctypes.POINTER(ctypes.c_double)
    g = B.Grid(32, 16, 8, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    ph = B.Phys(0.9, 0.72, 1.0, 1e-3, 1.0, 0.3, 1, 0, 0.1, 1.0, 0)  # gamma <= 1
    ctx = ctypes.c_void_p()
    st = lib.cdns_create(ctypes.byref(g), ctypes.byref(ph), 0, 1 << 20, 1 << 20, 1 << 40, None,
                         ctypes.byref(ctx))
    assert st == B.CDNS_EINVAL and not ctx.value
    ph = B.Phys(1.4, 0.72, 1.0, 1e-3, 1.0, 0.3, 1, 0, 0.1, 1.0, 0)
    st = lib.cdns_create(ctypes.byref(g), ctypes.byref(ph), 0, 1 << 20, 1 << 20, 10, None,
                         ctypes.byref(ctx))
    assert st == B.CDNS_ENOMEM


def test_product_has_no_cpu_fallback():
    """The package never imports the oracle and fails loudly without its library."""
    pkg = os.path.join(ROOT, "paper_2004_02276_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "cdns_oracle" not in txt, f
