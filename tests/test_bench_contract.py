"""Host-side contract of bench.py (no GPU): the multi-GPU refusal and the recorded
HBM traffic of the dominant kernel, which is reported only for the lattice and the
stencil source the counters were taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_recorded_traffic_only_for_its_lattice():
    import hashlib
    import re

    summary = open(os.path.join(ROOT, "profiles", "hop_f64_16x16x16x32_counters.md")).read()
    rec = json.loads(re.search(r"traffic_json: (\{.*\})", summary).group(1))
    src = open(os.path.join(ROOT, "paper_1805_09584_amd", "csrc", "kern_dslash.hip"), "rb").read()
    current = rec["source_sha256"] == hashlib.sha256(src).hexdigest()
    t = bench.recorded_traffic("hop_f64", (32, 16, 16, 16))
    # reported while the stencil source is the one the counters were taken on, null after
    # any change to it
    assert (t == rec["bytes_per_launch"]) if current else (t is None)
    assert bench.recorded_traffic("hop_f64", (64, 32, 32, 32)) is None
    assert bench.recorded_traffic("no_such_class", (32, 16, 16, 16)) is None
