"""Host-side behaviour of bench.py (no GPU): the one-GPU rule, the kernel
source hash that keys the committed counter figures, and the CPU baseline's
worker processes."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_kernel_source_hash_ignores_comments_and_host_code(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1901_02716_amd", "csrc")
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    # the same tree with a comment added to a kernel file and the host file changed
    fake = tmp_path / "paper_1901_02716_amd" / "csrc"
    fake.mkdir(parents=True)
    for name in os.listdir(src):
        text = open(os.path.join(src, name), encoding="utf-8").read()
        if name == "kernels_generic.hip":
            text = "// a comment\n" + text.replace("{", "{  /* another */", 1)
        if name == "maclab_api.hip":
            text += "\nint unused_host_symbol = 0;\n"
        (fake / name).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h
    (fake / "kernels_generic.hip").write_text((fake / "kernels_generic.hip").read_text() + "\nint x = 1;\n")
    assert bench.kernel_source_hash() != h


def test_committed_traffic_figures_are_keyed_by_the_hash():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, v in rec.items():
        assert set(v) >= {"bytes_per_launch", "fetch_bytes", "write_bytes", "source_hash"}, key
        assert v["bytes_per_launch"] == v["fetch_bytes"] + v["write_bytes"] or \
            abs(v["bytes_per_launch"] - v["fetch_bytes"] - v["write_bytes"]) <= 2
    assert bench.load_traffic("cube256", "fp32") in (None, rec["cube256:fp32"]["bytes_per_launch"])


def test_cpu_baseline_runs_oracle_workers():
    cores = bench.host_cores()
    assert 1 <= len(cores) <= 16
    mlups, slowest, secs = bench.cpu_baseline("cube64", 1, cores[:2])
    assert len(secs) == len(cores[:2]) and slowest == max(secs) > 0
    assert mlups == len(cores[:2]) * 62 ** 3 / slowest / 1e6
    assert bench.cpu_model()
