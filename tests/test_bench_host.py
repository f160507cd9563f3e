"""Host-side logic of the benchmark (no GPU): the counter-based HBM traffic
is reported only for the kernel source, workload and step window it was
taken on; the source key ignores comments and blank lines; the flop count
of the shock-capturing flux belongs to the current code."""
import json
import os

import bench


def test_traffic_keyed_to_source_and_workload(monkeypatch):
    with open(os.path.join(bench.ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    ent = t["k_weno"]
    st, wu = ent["steps"], ent["warmup"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: ent["source_hash"])
    assert bench.load_traffic("k_weno", ent["workload"], st, wu) == ent["hbm_bytes_per_launch"]
    assert bench.load_traffic("k_weno", "sbli", st, wu) is None        # other workload
    assert bench.load_traffic("k_weno", ent["workload"], st + 1, wu) is None  # other window
    assert bench.load_traffic("k_weno", ent["workload"], st, wu + 1) is None
    assert bench.load_traffic("k_nonexistent", ent["workload"], st, wu) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("k_weno", ent["workload"], st, wu) is None  # other source


def test_traffic_entries_per_workload(tmp_path, monkeypatch):
    """A kernel may carry one entry per workload (a list)."""
    t = {"k_rhs": [{"source_hash": "a" * 16, "workload": "channel", "steps": 20, "warmup": 5,
                    "hbm_bytes_per_launch": 1},
                   {"source_hash": "a" * 16, "workload": "sbli", "steps": 20, "warmup": 5,
                    "hbm_bytes_per_launch": 2}]}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(t))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "a" * 16)
    assert bench.load_traffic("k_rhs", "channel", 20, 5) == 1
    assert bench.load_traffic("k_rhs", "sbli", 20, 5) == 2
    assert bench.load_traffic("k_rhs", "bl", 20, 5) is None


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


def test_weno_flop_count_belongs_to_the_current_code():
    """The per-interface flop counts were taken from the shock-capturing flux
    code as it stands; a change there must come with a recount."""
    assert bench.weno_source_hash() == bench.WENO_FLOPS_SOURCE_HASH
    # totals from their parts: one node's quantities, Roe and constants, the
    # stencil nodes' projections, 5 fields, back-projection
    assert bench.WENO_FLOPS_BY_ORDER[5] == 15 + 47 + 6 * 38 + 5 * (2 * 5 * 2 + 2 * 61 + 7) + 26
    assert bench.WENO_FLOPS_BY_ORDER[3] == 15 + 47 + 4 * 38 + 5 * (2 * 3 * 2 + 2 * 17 + 7) + 26
    assert bench.WENO_FLOPS_BY_ORDER[7] == 15 + 47 + 8 * 38 + 5 * (2 * 7 * 2 + 2 * 141 + 7) + 26
