"""bench.py reports the committed HBM traffic only for the kernels that were profiled: the digest of the
built kernels' instructions must equal the one recorded with the counters."""
import json
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, isa):
    prof = tmp_path / "profiles"
    prof.mkdir(parents=True)
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if f.startswith("traffic_"):
            shutil.copy(os.path.join(ROOT, "profiles", f), prof / f)
    b = tmp_path / "paper_2408_05962_amd" / "_build"
    b.mkdir(parents=True)
    if isa is not None:
        (b / "device_isa.sha256").write_text(isa + "\n")
    return tmp_path


def test_traffic_follows_the_kernel_digest(tmp_path, monkeypatch):
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_hiccl_staged_six_collectives_16r_64MiB.json")))
    assert rec["device_isa_sha256"] and rec["traffic_bytes_per_launch"] > 0
    monkeypatch.setattr(bench, "ROOT", str(_tree(tmp_path / "same", rec["device_isa_sha256"])))
    assert bench.measured_traffic("staged", 0, 0) == round(rec["traffic_bytes_per_launch"])
    assert bench.measured_traffic("staged", 65536, 0) is None        # another launch configuration
    monkeypatch.setattr(bench, "ROOT", str(_tree(tmp_path / "changed", "0" * 64)))
    assert bench.measured_traffic("staged", 0, 0) is None
    monkeypatch.setattr(bench, "ROOT", str(_tree(tmp_path / "unbuilt", None)))
    assert bench.measured_traffic("staged", 0, 0) is None


def test_built_digest_against_the_profiles():
    """The built kernels are the profiled ones, or bench.py reports no traffic (a kernel change since the
    counters were taken is not an error, only a measurement to repeat)."""
    import bench
    digest = os.path.join(ROOT, "paper_2408_05962_amd", "_build", "device_isa.sha256")
    if not os.path.exists(digest):
        pytest.skip("library not built")
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_hiccl_staged_six_collectives_16r_64MiB.json")))
    same = open(digest).read().strip() == rec["device_isa_sha256"]
    assert (bench.measured_traffic("staged", 0, 0) is not None) == same
    if not same:
        pytest.skip("kernels changed since the committed counters were taken: traffic is reported as null")


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N above 1 prints one JSON line saying that this benchmark runs on one GPU and
    exits with status 2, before it touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
