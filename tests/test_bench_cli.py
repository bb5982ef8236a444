"""CPU checks of the benchmark's command line: more than one GPU is refused
with a message (this build measures one GPU), and the byte and operation
counts it reports agree with their stated breakdowns."""
import os
import subprocess
import sys

from tests.conftest import ROOT


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_reported_unit_counts():
    sys.path.insert(0, ROOT)
    import bench
    # FP32 deviation storage: 19 populations read and written, the 16-byte
    # solid and wall masks of each 64-node tile
    assert bench.bytes_per_node("f32dev") == 19 * 4 * 2 + 16 / 64
    assert bench.bytes_per_node("f64") == 19 * 8 * 2 + 16 / 64
    # dipole pair: separation 3, |r|^2 5, |r| 1, 3/(4 pi |r|^5) 3, three dot
    # products 15, 5 (m1.r)(m2.r)/|r|^2 3, bracket and scale 19, accumulate 3,
    # surface gap 1
    assert bench.FLOPS_PER_PAIR == 3 + 5 + 1 + 3 + 15 + 3 + 19 + 3 + 1
    assert len(bench.kernel_sha()) == 16


def test_launch_sample_stride():
    sys.path.insert(0, ROOT)
    import bench
    # odd strides (the pass alternates its workgroup order every step, so both
    # orders are sampled), about LAUNCH_SAMPLES launches per run
    for steps in (1, 5, 50, 100, 400, 1000, 2001):
        k = bench.sample_stride(steps)
        assert k % 2 == 1
        n = len(range(0, steps, k))
        assert 1 <= n <= steps
        if steps >= 2 * bench.LAUNCH_SAMPLES:
            assert bench.LAUNCH_SAMPLES // 2 <= n <= 2 * bench.LAUNCH_SAMPLES
    assert bench.sample_stride(1000) == 25
