"""Host logic of bench.py (no GPU): the argument contract, the algorithmic
byte count the roofline divides by, and the rule that stored traffic counters
apply only to the kernel sources they were measured on."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_several_gpus_are_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("args", [("--steps", "0"), ("--warmup", "-1")])
def test_bad_step_counts_are_refused(args):
    r = _run(*args)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_algorithmic_bytes_of_the_benchmark_batch():
    # 12 B per vertex (x, y, s in FP32), 37 B per segment, 10 B per path
    assert bench.algorithmic_bytes(69_591_158, 337_424, 4096) == 847_619_544


def test_stored_traffic_applies_only_to_its_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2007_00308_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("ps_kernels.hip", "ps_device.h"):
        shutil.copy(os.path.join(ROOT, "paper_2007_00308_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"source_sha256": bench.kernel_source_digest(), "emit_configs": {"1,7,4": 123}}
    (tmp_path / "profiles" / "emit_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("1,7,4") == 123
    assert bench.measured_traffic("1,8,4") is None
    with open(csrc / "ps_kernels.hip", "a") as fh:   # any change to the kernels
        fh.write("\n")
    assert bench.measured_traffic("1,7,4") is None
