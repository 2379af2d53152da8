"""The bench's counter table belongs to the kernel sources in the tree, and a
run on more than one GPU is refused with a message (host-only checks)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_counter_table_matches_the_kernel_sources():
    """every rocprofv3 figure in the table was taken on the kernel sources of
    this tree (a kernel change without new profiles would print stale
    traffic and VALU figures otherwise; the bench prints null for them)"""
    import bench
    h = bench.kernel_source_hash()
    assert bench.MEASURED
    assert {k[3] for k in bench.MEASURED} == {h}
    for (w, prec, tile, _), v in bench.MEASURED.items():
        assert prec in ("fp64", "mixed") and tile >= 0
        assert v["valu_per_cell_stage"] > 0 and v["traffic_bytes"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
