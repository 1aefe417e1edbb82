"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the benchmark measures one GPU), and the byte model the roofline divides
by matches the per-unit bytes stated for the kernels."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_byte_model():
    sys.path.insert(0, ROOT)
    import bench
    # per line unknown: cell 4 + lx, ly + chord [+ |beta| + load] + gathered + written value
    assert [bench.LINE_BYTES[k] for k in (("fp32", 0), ("fp32", 1), ("fp64", 0), ("fp64", 1))] == [32, 24, 60, 44]
    # per grid node: FP32 write / accumulate, FP64 write / update
    assert [bench.SCATTER_BYTES[k] for k in (("fp32", 2), ("fp32", 3), ("fp64", 2), ("fp64", 3))] == [50, 66, 118, 130]
