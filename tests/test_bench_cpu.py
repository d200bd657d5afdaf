"""bench.py's host logic on the CPU: the committed PMC summaries parse, their
figures are consistent, and a summary's traffic is used only while the
kernel sources it was taken on are the current ones."""
import glob
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summaries():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*__pmc.md"))):
        m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
        if m:
            out.append((os.path.basename(path), json.loads(m.group(1))))
    return out


def test_pmc_summaries_are_consistent():
    sums = _summaries()
    assert sums, "no PMC summaries under profiles/"
    for name, d in sums:
        assert name == f"{d['kernel']}__{d['workload']}__pmc.md", name
        assert re.fullmatch(r"[0-9a-f]{16}", d["src_hash"]), name
        hbm = d["fetch_kib_per_launch"] * 1024 * d["fetch_scale"] + d["write_kib_per_launch"] * 1024 * d["write_scale"]
        assert abs(hbm - d["hbm_bytes_per_launch"]) <= 1e-5 * hbm, name   # (stored figures are rounded)
        assert d["traffic_over_algorithmic"] == pytest.approx(d["hbm_bytes_per_launch"] / d["algorithmic_bytes_per_launch"],
                                                              abs=1e-4), name
        assert 0.9 < d["traffic_over_algorithmic"] < 1.5, name
        assert d["launches"] >= 1


def test_traffic_used_only_for_the_profiled_sources(monkeypatch):
    import bench
    name, d = _summaries()[0]
    monkeypatch.setattr(bench, "kernel_src_hash", lambda: d["src_hash"])
    assert bench.read_traffic(d["kernel"], d["workload"]) == d["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_src_hash", lambda: "0" * 16)
    assert bench.read_traffic(d["kernel"], d["workload"]) is None
    assert bench.read_traffic("k_none", d["workload"]) is None
