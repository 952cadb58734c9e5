"""bench.py's command-line contract, checked without a GPU: more than one
GPU is refused with a message, the sources that key the stored traffic
record exist, and the JSON line leads with the contract's fields."""
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


def test_line_leads_with_the_contract_fields():
    sys.path.insert(0, ROOT)
    import bench
    out = {"next_rows": {}, "roofline": {"frac": 0.4}, "value": 6.0, "metric": "m", "cpu_baseline": {"value": 0.01},
           "dslash": {}, "unit": "solves/s", "config": {"workload": "w"}, "fp64_time_to_1e10_ms": 437.0}
    keys = list(bench.ordered_line(out))
    assert keys[:3] == ["metric", "value", "unit"]
    assert keys.index("config") < keys.index("fp64_time_to_1e10_ms") < keys.index("roofline")
    assert keys.index("roofline") + 1 == keys.index("cpu_baseline")
    assert keys[-2:] == ["next_rows", "dslash"] and len(keys) == len(out)
