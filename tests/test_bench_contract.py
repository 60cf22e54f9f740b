"""CPU checks of the benchmark's bookkeeping (no GPU): the committed counter summary
of the r_{n+1} pass belongs to the current device code, so the bench reports its
measured traffic; and the benchmark refuses more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_summary_matches_current_device_code():
    """Any change to the stencil kernels must come with a fresh counter summary."""
    traffic, alg = bench.measured_traffic("medium_48x48x96", "fp64", 1, 18)
    assert traffic is not None, ("profiles/ traffic summary is stale: re-run the FETCH_SIZE / "
                                 "WRITE_SIZE passes for the current kernels.hpp")
    assert alg == 3 * 221184 * 16 * 64
    assert 1.0 <= traffic / alg < 2.0
    # another shape or workload gets no traffic figure
    assert bench.measured_traffic("medium_48x48x96", "fp64", 3, 18) == (None, None)
    assert bench.measured_traffic("tiny_16x16x24", "fp64", 1, 18) == (None, None)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
