"""bench.py's command line on the host (no GPU): more than one GPU is
refused with a message and exit status 2 before anything touches a
device, and the profile summaries it reads are recognised only for the
kernel sources they were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_profile_figures_follow_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # the committed summaries carry the hash of the current kernel sources
    assert bench.measured_traffic() is not None
    assert bench.measured_valu() is not None
    # a summary taken on other sources is ignored
    stale = tmp_path / "pmc.md"
    stale.write_text("kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_stage_launch: 1.0e8\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(stale))
    assert bench.measured_traffic() is None
