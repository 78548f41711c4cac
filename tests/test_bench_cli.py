"""bench.py on the CPU: the single-GPU contract and the committed profiles it
reads.

The HBM traffic the bench line reports comes from committed rocprofv3 counter
summaries, and only while the kernels' sources hash to the value those
counters were taken on: a kernel change without new counters would turn the
line's `traffic` fields into null, which this test catches.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_summaries_match_the_kernel_sources():
    import bench
    for kernel in ("k_dcgs_update", "k_precond_fused"):
        t = bench.read_traffic("bumps_8x8x8_p10", kernel)
        assert t is not None and t > 0, kernel


def test_profile_summaries_name_their_commands():
    prof = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(prof))
    assert names
    for n in names:
        text = open(os.path.join(prof, n)).read()
        assert "rocprofv3" in text, n
        assert "_work" not in text, n   # commands run committed files only
