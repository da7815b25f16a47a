"""Host-side checks of bench.py that need no GPU: more than one GPU is
refused before anything touches a device, and the CPU-only helpers of the
oracle baseline report what they measured."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_host_cpu_record():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert h["cores_available"] >= 1
    assert h["model"] is None or isinstance(h["model"], str)


def test_no_graphs_value_is_accepted_by_the_library():
    """--no-graphs sets the library's largest graph length, which every timed
    call stays below (so each step is a direct launch); ng_set_graph_steps
    accepts 1..4096."""
    sys.path.insert(0, ROOT)
    import bench
    assert 1 <= bench.NO_GRAPH_STEPS <= 4096
