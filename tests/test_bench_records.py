"""bench.py reports recorded HBM traffic only while the kernel sources still
hash to the value stored with the record."""
import os
import shutil

import bench


def _tree(tmp_path, body="kernel A"):
    root = tmp_path / "repo"
    (root / "paper_2506_08262_amd" / "csrc").mkdir(parents=True)
    (root / "include").mkdir()
    (root / "profiles").mkdir()
    (root / "paper_2506_08262_amd" / "csrc" / "k.hip").write_text(body)
    (root / "include" / "rrs.h").write_text("header")
    return root


def test_record_used_only_while_sources_match(tmp_path, monkeypatch):
    root = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.kernel_sources_hash()
    (root / "profiles" / "k_select_c2.md").write_text(
        "# summary\n\ntraffic-record: kernel=k_select workload=c2 precision=f32 "
        f"sources={h} fetch_bytes=1.5e10 write_bytes=2e6\n")
    rec = bench.recorded_traffic("k_select", "c2", "f32")
    assert rec["bytes"] == 1.5e10 + 2e6 and rec["record"] == "profiles/k_select_c2.md"
    assert bench.recorded_traffic("k_select", "c2", "bf16") is None
    assert bench.recorded_traffic("k_gemm", "c2", "f32") is None
    # any change to a kernel source invalidates the record
    (root / "paper_2506_08262_amd" / "csrc" / "k.hip").write_text("kernel B")
    assert bench.kernel_sources_hash() != h
    assert bench.recorded_traffic("k_select", "c2", "f32") is None


def test_committed_records_parse():
    """The summaries under profiles/ carry well-formed records (their hash may
    or may not match the working tree)."""
    pdir = os.path.join(os.path.dirname(bench.__file__), "profiles")
    n = 0
    for f in os.listdir(pdir):
        for ln in open(os.path.join(pdir, f)):
            if ln.startswith("traffic-record:"):
                kv = dict(t.split("=", 1) for t in ln.split(":", 1)[1].split() if "=" in t)
                assert {"kernel", "workload", "precision", "sources", "fetch_bytes",
                        "write_bytes"} <= set(kv)
                assert float(kv["fetch_bytes"]) > 0
                n += 1
    assert n >= 1
