"""Host-side checks of bench.py that need no GPU: more than one GPU is
refused before anything touches a device, the CPU-only helpers of the
oracle baseline report what they measured, and the profile summaries read
their traces as stated."""
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


def test_profile_summary_of_cooperative_launches(tmp_path):
    """The cooperative-launch summary takes, per run, the longest launch of the
    named kernel with the given workgroup count and divides it by the steps
    it ran; a run with no such launch is an error."""
    import pytest
    sys.path.insert(0, ROOT)
    from paper_1805_03442_amd import profiling
    head = "Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X,Workgroup_Size_X\n"
    rows = ['"void ng::run_coop1d_kernel<ng::Dev32<4>, 2>(int)",0,260000,196608,768',
            '"void ng::run_coop1d_kernel<ng::Dev32<4>, 2>(int)",0,240000000,196608,768',
            '"void ng::run_coop1d_kernel<ng::Plain64<4>, 1>(int)",0,11000000,1280,256',
            '"void ng::run_coop1d_kernel<ng::Plain64<4>, 1>(int)",0,800000000,131072,512']
    trace = tmp_path / "trace.csv"
    trace.write_text(head + "\n".join(rows) + "\n")
    md = profiling.coop_markdown(str(trace), "cmd", ["Dev32<4>:20000:256:a",
                                                     "Plain64<4>:2000:5:b"], None)
    assert "| a | `ng::run_coop1d_kernel<ng::Dev32<4>, 2>` | 256 x 768 | 240000.0 | 20000 | 12.00 |" in md
    assert "| b | `ng::run_coop1d_kernel<ng::Plain64<4>, 1>` | 5 x 256 | 11000.0 | 2000 | 5.50 |" in md
    with pytest.raises(SystemExit):
        profiling.coop_markdown(str(trace), "cmd", ["Mix32<4>:10:256:c"], None)
