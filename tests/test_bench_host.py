"""Host logic of bench.py that needs no GPU: the stored HBM traffic is only
reported while the kernel, executor and task-graph sources still match the
SHA-256s recorded with the counters, and the multi-GPU request is refused."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record(tmp_path, shas, value=12345):
    p = tmp_path / "profile.md"
    rec = {"kernel": "dc_gemm_kernel", "source_sha256s": shas, "bytes_per_launch": value}
    p.write_text("# summary\n\ntraffic: " + json.dumps(rec) + "\n")
    return str(p)


def _sha(rel):
    return hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()


def test_stored_traffic_follows_source_hashes(tmp_path, monkeypatch):
    srcs = ["paper_1304_0878_amd/csrc/gemm_kernel.hip", "paper_1304_0878_amd/csrc/runtime.cpp",
            "paper_1304_0878_amd/csrc/highlevel.cpp"]
    good = {s: _sha(s) for s in srcs}
    monkeypatch.setattr(bench, "PROFILE", _record(tmp_path, good))
    assert bench.stored_traffic(32768, 512) == 12345
    assert bench.stored_traffic(8192, 512) is None          # another workload
    for s in srcs:                                          # any one source changed
        bad = dict(good)
        bad[s] = "0" * 64
        monkeypatch.setattr(bench, "PROFILE", _record(tmp_path, bad))
        assert bench.stored_traffic(32768, 512) is None
    monkeypatch.setattr(bench, "PROFILE", _record(tmp_path, {}))
    assert bench.stored_traffic(32768, 512) is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode != 0 and "single-GPU" in (r.stdout + r.stderr)
