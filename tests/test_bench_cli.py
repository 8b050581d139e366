"""Host-side checks of the benchmark script: it refuses more than one GPU with
a message, and it reads the counter record only for a matching workload and
kernel-source hash (no GPU is touched)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _record(tmp_path, workload, sha):
    p = tmp_path / "counters.txt"
    p.write_text("# header: ignored\n\n"
                 f"workload: {workload}\nkernel_sources_sha256: {sha}\ntraffic_bytes_per_launch: 123\n"
                 "hbm_gbs: 4\nmfma_util: 0.5\n\n"
                 f"workload: other\nkernel_sources_sha256: {sha}\ntraffic_bytes_per_launch: 9\n")
    return str(p)


def test_counter_record_lookup(tmp_path, monkeypatch):
    w = "c3 fp64 samples=16 chi=64 chi_x=64 cutoff=0 env=yes"
    monkeypatch.setattr(bench, "COUNTER_FILE", _record(tmp_path, w, bench.kernel_hash()))
    kv = bench.stored_counters(w)
    assert kv["traffic_bytes_per_launch"] == "123" and kv["mfma_util"] == "0.5"
    assert bench.stored_counters("c3 fp32 samples=16 chi=64 chi_x=64 cutoff=0 env=yes") == {}


def test_counter_record_ignored_after_kernel_change(tmp_path, monkeypatch):
    w = "c3 fp64 samples=16 chi=64 chi_x=64 cutoff=0 env=yes"
    monkeypatch.setattr(bench, "COUNTER_FILE", _record(tmp_path, w, "0" * 64))
    assert bench.stored_counters(w) == {}


def test_committed_record_parses():
    with open(bench.COUNTER_FILE) as f:
        blocks = [b for b in f.read().split("\n\n") if "workload:" in b]
    assert blocks
    for b in blocks:
        kv = dict(l.split(":", 1) for l in b.splitlines() if ":" in l and not l.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        assert len(kv["kernel_sources_sha256"]) == 64
        assert float(kv["traffic_bytes_per_launch"]) > float(kv["algorithmic_bytes_per_unmasked_launch"]) > 0
        assert 0 < float(kv["mfma_util"]) <= 1
