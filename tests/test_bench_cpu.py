"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
report-section filter (CPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_unknown_report_section_is_refused():
    r = _bench("--report", "--sections", "training,bogus")
    assert r.returncode == 2
    assert "unknown report sections ['bogus']" in r.stderr


def test_empty_report_section_list_runs_nothing():
    r = _bench("--report", "--sections", "")
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == ""
