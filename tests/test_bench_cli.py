"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the library is measured on one GPU), and the profile that supplies
the measured traffic of the headline kernel parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_profile_parses():
    sys.path.insert(0, ROOT)
    import bench
    traffic, note = bench.measured_traffic()
    # either the counters match the current solve sources, or the field is
    # withheld with a reason
    assert (traffic is None and note) or (traffic > 0 and int(note) > 0)
