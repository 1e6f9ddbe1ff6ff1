"""Host-side checks of bench.py's command line (no GPU): a request for more than
one GPU is refused with a message and exit status 2, before anything touches a
device, and every workload name parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("window", "large", "uneven", "at", "coupling", "coupling_paper", "rates"):
        assert w in r.stdout
    for opt in ("--uneven-schedule", "--large-integrator", "--adjoint-layout"):
        assert opt in r.stdout
