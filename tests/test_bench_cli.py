"""The benchmark's command line on the CPU: a request for more than one GPU
ends at once with exit status 2 and a message (the solve of one object is
not sharded), before anything touches a device; and the committed HBM
traffic record names the sources it was measured on: the GEMM kernel and
the scheduler that forms its launches."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_names_its_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_zgemm_traffic_sphere_ka20_49152_mixed.json")))
    assert set(rec["source_sha256"]) == {"paper_2408_17116_amd/csrc/batch.hip", "paper_2408_17116_amd/csrc/hmat.hip"}
    assert rec["traffic_bytes_per_launch"] > 0
