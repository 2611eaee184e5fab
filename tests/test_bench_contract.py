"""The benchmark script's command-line contract, on the CPU: more than one GPU
is refused with a JSON error line and exit status 2, and the recorded HBM
traffic table names kernels the bench times."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_table_names_timed_kernels():
    import bench
    timed = {bench.KERNEL_NAMES.get(k, f"k_{k}") for k in bench.KERNEL_FILES}
    for workload, table in bench.MEASURED_TRAFFIC.items():
        assert workload in bench.WORKLOADS
        for kname, rec in table.items():
            assert kname in timed
            assert len(rec["src"]) == 16 and rec["bytes"] > 0
    # every timed kernel's source hash can be taken
    for k in bench.KERNEL_FILES:
        assert len(bench.kernel_source_hash(k)) == 16
