"""bench.py's command-line contract on the CPU: more than one GPU is refused with a message,
and the traffic table it keeps is well formed (one entry per tile shape it may report)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_table_is_well_formed():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.pop(0)
    T = bench.TRAFFIC
    assert T["kernel"] in bench.FLOPS_PER_POINT
    assert len(T["source_sha"]) == 64
    for shape, nbytes in T["bytes"].items():
        assert len(shape) == 2 and all(isinstance(v, int) for v in shape)
        # at least t, y and the stored tree of N = 2^20 points, at most a few times that
        assert 70e6 < nbytes < 400e6
