"""The benchmark's command-line contract on the CPU: more than one GPU is refused before
anything touches a GPU, and the host-description helpers return plain data."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_host_description_helpers():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert set(h) == {"model", "logical_cpus"} and h["logical_cpus"] >= 1
    clocks = bench.gpu_clocks()
    assert clocks is None or all(isinstance(x, str) and "clk" in x for x in clocks)
