"""bench.py's command line on the host: more than one GPU is refused with a
message and exit status 2, before any device is touched."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_counter_figures_match_the_kernel_sources():
    """The committed traffic and instruction counts were taken on the current
    kernel sources (bench.py drops a figure whose digest does not match)."""
    import json

    sys.path.insert(0, ROOT)
    import bench

    for name in ("traffic_c1.json", "valu_c1.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            rec = json.load(f)
        assert rec["source_digest"] == bench.source_digest(), name
    with open(os.path.join(ROOT, "profiles", "valu_c1.json")) as f:
        v = json.load(f)
    # 16,384,000 evaluations in chunks of 64: about a hundred vector instructions per chunk
    assert 50 < v["valu_wave_insts_per_launch"] / (16384000 / 64) < 200
