"""CPU checks of the benchmark's bookkeeping (no GPU): the committed counter summary
of the r_{n+1} pass belongs to the current device code, so the bench reports its
measured traffic; and the benchmark refuses more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary_fields():
    with open(bench.TRAFFIC_FILE) as fh:
        kv = dict(l.split(":", 1) for l in fh if ":" in l and not l.startswith("#"))
    return {k.strip(): v.strip() for k, v in kv.items()}


def test_traffic_summary_matches_current_device_code():
    """Any change to the stencil kernels must come with a fresh counter summary; the
    bench reports traffic only for the workload, precision and launch shape it names."""
    kv = _summary_fields()
    wl, prec, tile, zc = kv["workload"], kv["precision"], int(kv["tile"]), int(kv["zchunk"])
    traffic, alg = bench.measured_traffic(wl, prec, tile, zc)
    assert traffic is not None, ("profiles/ traffic summary is stale: re-run the FETCH_SIZE / "
                                 "WRITE_SIZE passes for the current kernels.hpp")
    assert wl == "medium_48x48x96" and prec == "fp64"
    assert alg == 3 * 221184 * 16 * 64  # every column block active in the counted launches
    assert 1.0 <= traffic / alg < 2.0
    # another shape or workload gets no traffic figure
    assert bench.measured_traffic(wl, prec, tile % 4 + 1, zc) == (None, None)
    assert bench.measured_traffic(wl, prec, tile, zc + 1) == (None, None)
    assert bench.measured_traffic("tiny_16x16x24", prec, tile, zc) == (None, None)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
