"""CPU checks of the benchmark's bookkeeping (no GPU): the committed counter summary
of the r_{n+1} pass belongs to the current device code, so the bench reports its
measured traffic; and the benchmark refuses more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_summary_matches_current_device_code():
    """Any change to the stencil kernels must come with a fresh counter summary; the
    bench reports traffic only for the workload, precision and launch shapes it names
    (one record per shape the autotuner picks on the medium workload)."""
    recs = bench.traffic_records()
    assert len(recs) >= 1
    shapes = {(int(kv["tile"]), int(kv["zchunk"]), int(kv.get("cache_mode", 0))) for kv in recs}
    assert len(shapes) == len(recs)  # no shape twice
    for kv in recs:
        wl, prec, tile, zc = kv["workload"], kv["precision"], int(kv["tile"]), int(kv["zchunk"])
        cm = int(kv.get("cache_mode", 0))
        traffic, alg = bench.measured_traffic(wl, prec, tile, zc, cm)
        assert traffic is not None, ("profiles/ traffic summary is stale: re-run the "
                                     "FETCH_SIZE / WRITE_SIZE passes for the current kernels.hpp")
        assert wl == "medium_48x48x96" and prec == "fp64"
        assert alg == 3 * 221184 * 16 * 64  # every column block active in the counted launches
        assert 1.0 <= traffic / alg < 2.0
        # another shape or workload gets no traffic figure
        for other in ((tile % 4 + 1, zc, cm), (tile, zc + 1, cm), (tile, zc, (cm + 1) % 3)):
            if other not in shapes:
                assert bench.measured_traffic(wl, prec, *other) == (None, None)
        assert bench.measured_traffic("tiny_16x16x24", prec, tile, zc, cm) == (None, None)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_recorded_tuning_is_in_the_library_format_and_has_a_traffic_record():
    """The bench's recorded launch shape for the medium workload is a line the library
    reads (its exact record form, values in range), and the counter summary covers it."""
    import json
    import re
    with open(bench.TUNE_RECORDS) as fh:
        lines = [l.rstrip("\n") for l in fh if l.strip()]
    form = re.compile(
        r'\{"arch": "gfx\w+", "precision": "(fp64|mixed)", "grid": \[\d+, \d+, \d+\], '
        r'"nf": \d, "atoms": \d+, "block_width": \d+, "blocks": \d+, "energies": \d+, '
        r'"rows": \d+, "tile": [1-4], "zchunk": \d+, "shift_chunk": (1|4|16), '
        r'"cache_mode": [0-2], "zchunk_mu": \d+\}$')
    assert lines and all(form.match(l) for l in lines)
    recs = [json.loads(l) for l in lines]
    med = [r for r in recs if r["grid"] == [48, 48, 96] and r["precision"] == "fp64"]
    assert len(med) == 1
    r = med[0]
    assert (r["nf"], r["atoms"], r["block_width"], r["blocks"], r["energies"], r["rows"]) == \
        (4, 40, 8, 8, 128, 64)
    assert 1 <= r["zchunk"] <= 96 and 0 <= r["zchunk_mu"] <= 96
    traffic, _ = bench.measured_traffic("medium_48x48x96", "fp64", r["tile"], r["zchunk"],
                                        r["cache_mode"])
    assert traffic is not None
