"""bench.py's command line on the CPU: it measures one GPU only, so a
request for more exits with a message and a non-zero status before touching
any device; the traffic lookup finds nothing for a kernel or a source hash
it has no counters for."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_traffic_lookup_and_source_hash():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert bench.measured_traffic("no_such_kernel", "c1") is None
