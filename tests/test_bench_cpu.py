"""Host-side checks of the benchmark's contract (no GPU): it measures one GPU and
refuses several, and the committed counter summary it reads `roofline.traffic`
from has the expected form."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    """--gpus above 1 exits with status 2 and a message, before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, r.stderr
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in msg["error"]


def test_traffic_record_form():
    """The step profile ends with one traffic-json record: measured bytes per launch
    of every pass, for each schedule the autotuner picks between, and the hash of
    the kernel sources they were taken from."""
    lines = open(os.path.join(ROOT, "profiles", "step_256_fp32_k3.md")).read().splitlines()
    recs = [json.loads(ln[len("traffic-json: "):]) for ln in lines if ln.startswith("traffic-json: ")]
    assert len(recs) == 1
    rec = recs[0]
    assert len(rec["sources_sha256"]) == 64
    assert set(rec["bytes"]) >= {"2", "4"}
    for per_pass in rec["bytes"].values():
        for k in ("k_plane_fwd", "k_columns", "k_plane_inv", "k_project_gram"):
            assert per_pass[k] > 1e8  # hundreds of MB per launch at 256^3, three states
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("k_plane_inv", 3) is None  # no record for that schedule
