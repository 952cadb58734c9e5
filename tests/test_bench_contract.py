"""bench.py's command-line contract, checked without a GPU: more than one
GPU is refused with a message, and the sources that key the stored traffic
record exist."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_sources_exist():
    sys.path.insert(0, ROOT)
    import bench
    csrc = os.path.join(ROOT, "paper_2112_00501_amd", "csrc")
    for name in bench.SAP_KERNEL_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    assert len(bench.source_hash(bench.SAP_KERNEL_SOURCES)) == 16
