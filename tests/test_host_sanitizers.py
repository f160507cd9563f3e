"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle, built with gcc -fsanitize=address,undefined, runs every entry
  point on small problems of each boundary set-up (periodic, walls with
  forcing, inflow / outflow / imposed shock, digital-filter inflow) and
  scheme order in a child process with the sanitizer runtime preloaded; any
  report aborts the child.
* The library's host glue (argument checks, workspace layout, boundary
  parameter expansion of cdns_api.hip), built with the host part under
  both sanitizers, runs the entry points that need no GPU.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    "OMP_NUM_THREADS": "2",
}


def _run_child(script, preload, tmp_path):
    path = tmp_path / "child.py"
    path.write_text(textwrap.dedent(script))
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload, PYTHONPATH=ROOT)
    res = subprocess.run([sys.executable, str(path)], env=env, capture_output=True, text=True,
                         timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc AddressSanitizer runtime not available")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-std=c11",
                    "-fPIC", "-shared", "-o", str(lib), os.path.join(ROOT, "oracle", "cdns_oracle.c"),
                    "-lm"], check=True)
    script = f"""
    import dataclasses
    import numpy as np
    import oracle
    import problems as P
    oracle._LIB = {str(lib)!r}
    def run(pr, steps=1):
        r, th, nf, ifl, f = oracle.rhs(pr, want_flags=True)
        dt = oracle.dt(pr)
        w = oracle.advance(pr, steps, dt_fixed=dt)
        oracle.advance(pr, 1, cfl=pr.cfl)
        oracle.totals(pr, w)
        oracle.extrema(pr, w)
        acc = oracle.stats(pr, w)
        oracle.stats_means(pr, acc, 1)
        oracle.stats_means(pr, acc, 1, average_x=True)
        for d in range(3):
            oracle.iface_flux(pr, d)
        if pr.bcs[2][0] != P.BC_PERIODIC:
            oracle.ghosts_y(pr, 2)
            oracle.ghosts_y(pr, 3)
        oracle.lf_alpha(pr, 0, 2, 2, 2)
        assert np.isfinite(r).all() and np.isfinite(w).all()
    run(P.taylor_green(8))
    run(P.small_channel(12, 10, 8), 2)
    run(P.small_sbli(24, 16, 6), 2)
    bl = P.small_boundary_layer(16, 12, 8)
    run(bl, 2)
    oracle.df_coeffs(bl)
    psi, plane, fl = oracle.df_update(bl, 0, 0.0, True)
    oracle.df_update(bl, 1, 1e-3, False, psi)
    for co, wo in ((2, 3), (6, 7)):
        run(dataclasses.replace(P.decaying_turbulence(12, mach=0.8, re=500.0, seed=3),
                                central_order=co, weno_order=wo))
    for r_ in (2, 3, 4):
        oracle.weno(r_, np.linspace(0.0, 1.0, 2 * r_ - 1))
        oracle.weno_parts(r_, np.linspace(0.0, 1.0, 2 * r_ - 1))
    oracle.eigenvectors(1.4, 1, 0.3, -0.2, 0.1, 3.0)
    oracle.rk_stage(np.ones(8), np.ones(8), np.ones(8), 0.1, 1)
    oracle.splitmix64(7, 3)
    print("oracle sanitized run ok", flush=True)
    """
    out = _run_child(script, asan, tmp_path)
    assert "oracle sanitized run ok" in out


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_library_host_glue_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    rt = _clang_asan_runtime()
    hipcc = "/opt/rocm/bin/hipcc"
    if rt is None or not os.path.exists(hipcc):
        pytest.skip("hipcc or clang AddressSanitizer runtime not available")
    csrc = os.path.join(ROOT, "paper_2004_02276_amd", "csrc")
    base = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]
    objs = []
    for src, san in (("cdns_api.hip", True), ("cdns_batch.hip", True), ("cdns_kernels.hip", False)):
        obj = tmp_path / src.replace(".hip", ".o")
        prebuilt = os.path.join(ROOT, "paper_2004_02276_amd", "_build", src.replace(".hip", ".o"))
        if not san and os.path.exists(prebuilt) and \
                os.path.getmtime(prebuilt) >= os.path.getmtime(os.path.join(csrc, src)):
            objs.append(prebuilt)     # device code and launchers: the regular build
            continue
        flags = (["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"] if san else [])
        subprocess.run([hipcc] + base + flags + ["-c", os.path.join(csrc, src), "-o", str(obj)],
                       check=True, capture_output=True)
        objs.append(str(obj))
    lib = tmp_path / "libcdns_san.so"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-shared-libsan", "-o", str(lib)] + objs, check=True, capture_output=True)
    script = f"""
    import ctypes
    import numpy as np
    from paper_2004_02276_amd import _binding as B
    B.LIB_PATH = {str(lib)!r}
    lib = B.load()
    assert b"gfx950" in lib.cdns_version()
    dp = ctypes.POINTER(ctypes.c_double)
    ye = np.full(16, 2.0); yee = np.zeros(16)
    for dims in ((32, 16, 8), (4, 16, 4), (3, 16, 8), (1 << 20, 16, 1 << 12)):
        g = B.Grid(dims[0], 16, dims[2], 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
        for prec in (0, 1, 5):
            lib.cdns_workspace_bytes(ctypes.byref(g), prec)
    lib.cdns_workspace_bytes(None, 0)
    g = B.Grid(32, 16, 8, 1.0, 1.0, ye.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    ok = B.Phys(1.4, 0.72, 1.0, 1e-3, 1.0, 0.3, 1, 1, 0.1, 1.0, 0)
    bad = B.Phys(0.9, 0.72, 1.0, 1e-3, 1.0, 0.3, 1, 0, 0.1, 1.0, 0)
    ctx = ctypes.c_void_p()
    need = lib.cdns_workspace_bytes(ctypes.byref(g), 0)
    cases = [(None, ok, 0, 1 << 20, 1 << 20, need), (g, None, 0, 1 << 20, 1 << 20, need),
             (g, bad, 0, 1 << 20, 1 << 20, need), (g, ok, 3, 1 << 20, 1 << 20, need),
             (g, ok, 0, 1 << 20, (1 << 20) + 8, need), (g, ok, 0, 1 << 20, 1 << 20, need - 1),
             (g, ok, 0, 0, 1 << 20, need), (g, ok, 0, 1 << 20, 0, need)]
    for gg, ph, prec, st, ws, nb in cases:
        rc = lib.cdns_create(ctypes.byref(gg) if gg else None, ctypes.byref(ph) if ph else None,
                             prec, st, ws, nb, None, ctypes.byref(ctx))
        assert rc in (B.CDNS_EINVAL, B.CDNS_ENOMEM), rc
    ye_bad = np.array([2.0] * 15 + [-1.0])
    g2 = B.Grid(32, 16, 8, 1.0, 1.0, ye_bad.ctypes.data_as(dp), yee.ctypes.data_as(dp))
    assert lib.cdns_create(ctypes.byref(g2), ctypes.byref(ok), 0, 1 << 20, 1 << 20, need, None,
                           ctypes.byref(ctx)) == B.CDNS_EINVAL
    assert lib.cdns_create(ctypes.byref(g), ctypes.byref(ok), 0, 1 << 20, 1 << 20, need, None,
                           None) == B.CDNS_EINVAL
    for fn in ("cdns_rhs", "cdns_rk_step", "cdns_advance_n", "cdns_diagnostics",
               "cdns_diagnostics_noalloc", "cdns_stats_means", "cdns_destroy"):
        getattr(lib, fn).restype = ctypes.c_int32
    assert lib.cdns_rhs(None, 1, 1) == B.CDNS_EINVAL
    assert lib.cdns_rk_step(None, 0.5, 0.0) == B.CDNS_EINVAL
    assert lib.cdns_advance_n(None, 1, 0.5, 0.0) == B.CDNS_EINVAL
    assert lib.cdns_diagnostics(None, None) == B.CDNS_EINVAL
    assert lib.cdns_diagnostics_noalloc(None, None, None) == B.CDNS_EINVAL
    assert lib.cdns_stats_means(None, 0, None) == B.CDNS_EINVAL
    assert lib.cdns_destroy(None) == B.CDNS_EINVAL
    assert lib.cdns_last_error(None) == b"null context"
    assert lib.cdns_batch_workspace_bytes(0) == 0 and lib.cdns_batch_workspace_bytes(4) > 0
    print("library host glue sanitized run ok", flush=True)
    """
    out = _run_child(script, rt, tmp_path)
    assert "library host glue sanitized run ok" in out
