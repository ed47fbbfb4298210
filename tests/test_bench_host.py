"""Host logic of the benchmark and the profile summaries (no GPU needed).

* The HBM traffic a bench line reports comes from profiles/boxcar_traffic.json
  only while the kernel sources still hash to what the counters were taken
  on; the bench and the profile summariser must hash the same files the same
  way.
* More than one GPU is refused with a message.
* The oracle baseline sizes its row sample from a pilot.
"""
import json
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1611_09704_amd import profiling  # noqa: E402


@pytest.mark.parametrize("files", [bench.BOXCAR_SOURCES, bench.CLUSTER_SOURCES, bench.DEDISP_SOURCES])
def test_bench_and_summaries_hash_the_same_sources(files):
    assert bench.kernel_source_sha(files) == profiling.kernel_source_sha(files)


def test_source_sets_hash_differently():
    shas = {bench.kernel_source_sha(f) for f in (bench.BOXCAR_SOURCES, bench.CLUSTER_SOURCES, bench.DEDISP_SOURCES)}
    assert len(shas) == 3


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"kernel_sha": bench.kernel_source_sha(), "hbm_bytes_per_launch": 123.0}
    (prof / "boxcar_traffic.json").write_text(json.dumps({
        "ska": entry,
        "ska16": dict(entry, kernel_sha="0000000000000000"),
        "dedisp": {"kernel_sha": bench.kernel_source_sha(bench.DEDISP_SOURCES), "hbm_bytes_per_launch": 7.0},
    }))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_source_sha reads the sources under ROOT: keep it on the real tree
    monkeypatch.setattr(bench, "kernel_source_sha",
                        lambda files=bench.BOXCAR_SOURCES: profiling.kernel_source_sha(files))
    assert bench.load_traffic("ska") == 123.0
    assert bench.load_traffic("ska16") is None          # counters taken on other sources
    assert bench.load_traffic("dit") is None            # never measured
    assert bench.load_traffic("dedisp") == 7.0          # gated on its own source
    (prof / "boxcar_traffic.json").write_text("{not json")
    assert bench.load_traffic("ska") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_oracle_baseline_sizes_its_sample():
    x = torch.randn(12, 6000)
    out = bench.oracle_rows_baseline(x, list(range(1, 9)), "sqrtn", 0.5, label=", test")
    assert out["kind"] == "oracle" and out["unit"] == "GSamples/s" and out["cores"] >= 1
    assert 2 <= out["rows"] <= 12 and out["value"] > 0
    assert out["sample"].startswith("%d of 12 rows x 6000 samples, test" % out["rows"])
