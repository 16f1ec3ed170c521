"""bench.py reads roofline.traffic from a committed counter summary only while
the kernel source still has the hash the counters were taken on."""
import hashlib
import os

import bench


def _tree(tmp_path, src_text, sha):
    csrc = tmp_path / "paper_2305_17111_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text(src_text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_traffic.md").write_text(
        "# summary\n\nsome prose: with a colon\n\n"
        "source: paper_2305_17111_amd/csrc/k.hip\n"
        f"source_sha256: {sha}\n"
        "fetch_bytes_per_launch: 1.5e+09\n"
        "write_bytes_per_launch: 8.1e+07\n")


def test_traffic_read_while_source_unchanged(tmp_path, monkeypatch):
    text = "__global__ void k() {}\n"
    _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t, src = bench.measured_traffic("k_traffic.md", "k.hip")
    assert t == {"fetch": 1.5e9, "write": 8.1e7} and src == "k_traffic.md"


def test_traffic_null_once_source_changed(tmp_path, monkeypatch):
    _tree(tmp_path, "__global__ void k() { /* changed */ }\n",
          hashlib.sha256(b"__global__ void k() {}\n").hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t, why = bench.measured_traffic("k_traffic.md", "k.hip")
    assert t is None and "changed" in why


def test_committed_profiles_parse():
    """Every committed traffic summary carries the keys bench.py reads."""
    d = os.path.join(bench.ROOT, "profiles")
    for name in os.listdir(d):
        if name.endswith("_hbm_traffic.md"):
            text = open(os.path.join(d, name)).read()
            for key in ("source_sha256:", "fetch_bytes_per_launch:", "write_bytes_per_launch:"):
                assert key in text, (name, key)
