"""Host-side checks of the benchmark script (no GPU): more than one GPU is refused with a
message before anything touches a device, and every committed profile summary states
the rocprofv3 command that produced it."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_summaries_name_their_command():
    d = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(d) if f.endswith((".txt", ".md")))
    assert names
    for f in names:
        text = open(os.path.join(d, f)).read()
        assert "rocprofv3 " in text and " -- python -u bench.py" in text, f
