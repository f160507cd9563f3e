"""Host-side logic of the benchmark (no GPU): the counter-based HBM traffic
is reported only for the kernel source and the workload it was taken on,
and the source key ignores comments and blank lines."""
import json
import os

import bench


def test_traffic_keyed_to_source_and_workload(monkeypatch):
    with open(os.path.join(bench.ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    ent = t["k_weno"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: ent["source_hash"])
    assert bench.load_traffic("k_weno", ent["workload"]) == ent["hbm_bytes_per_launch"]
    assert bench.load_traffic("k_weno", "sbli") is None       # other workload
    assert bench.load_traffic("k_nonexistent", ent["workload"]) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("k_weno", ent["workload"]) is None  # other source


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_2004_02276_amd", "csrc", "cdns_kernels.hip")
    h0 = bench.kernel_source_hash()
    assert len(h0) == 16 and h0 == bench.kernel_source_hash()
    with open(src) as fh:
        text = fh.read()
    # the same code with an extra comment line and blank line hashes the same
    alt = tmp_path / "cdns_kernels.hip"
    alt.write_text("// a comment\n\n" + text)
    real_open = open

    def fake_open(path, *a, **k):
        return real_open(alt if os.path.abspath(str(path)) == src else path, *a, **k)

    monkeypatch.setattr("builtins.open", fake_open)
    assert bench.kernel_source_hash() == h0
