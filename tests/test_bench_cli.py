"""bench.py on the CPU: the single-GPU benchmark refuses a multi-GPU request with a message and
exit status 2, before touching torch or the GPU; counter-derived figures are tied to the kernel
source they were measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_profile_figures_are_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    """bench.py takes a kernel's HBM and LDS bytes from the committed counter summaries only
    while the kernel's source file still has the hash recorded with the counters."""
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.source_sha("splat_backward")
    traffic = tmp_path / "hbm.txt"
    traffic.write_text("# kernel launches fetch_KiB write_KiB bytes source_sha\n"
                       f"splat_backward 27 1.0 2.0 4275281439 {sha}\n"
                       "splat_forward 27 1.0 2.0 6886917464 0123456789abcdef\n")
    lds = tmp_path / "lds.txt"
    lds.write_text(f"splat_backward 27 1 2 57261195309 19674.2 32.0 0.2182 {sha}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(bench, "LDS_FILE", str(lds))
    assert bench.measured_traffic("splat_backward") == 4275281439.0
    assert bench.measured_traffic("splat_forward") is None      # recorded for another source
    assert bench.measured_traffic("trace") is None              # not in the summary
    assert bench.measured_lds("splat_backward") == 57261195309.0
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("splat_backward") is None
