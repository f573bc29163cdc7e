"""bench.py's command-line contract on the host: more than one GPU is refused
with a message (the library runs on one GPU), and the measured-traffic entry
names a source file that exists."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_traffic_entry_names_an_existing_kernel_source():
    sys.path.insert(0, ROOT)
    import bench
    assert os.path.exists(os.path.join(ROOT, "paper_2203_11154_amd", "csrc", bench.MEASURED_TRAFFIC["source"]))
    assert len(bench.kernel_source_hash(bench.MEASURED_TRAFFIC["source"])) == 16
    per_workload = bench.MEASURED_TRAFFIC["bytes_per_launch"]
    assert per_workload and all(set(v) <= {1, 2} and all(b > 0 for b in v.values()) for v in per_workload.values())
