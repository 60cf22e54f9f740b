"""The persistent autotuning records (SCOCG_TUNE_CACHE): a tuned launch shape is
written as one JSON line keyed by architecture, precision and problem shape; a fresh
handle of the same shape takes it without trials and gives the same columns bit for
bit; a record whose values are out of range is ignored."""
import json
import time

import numpy as np
import pytest

from paper_1502_00081_amd import scocg
from paper_1502_00081_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A = scocg.AUTO


def solve_auto(p):
    h = scocg.create_from_problem(p, precision=scocg.FP64)
    try:
        rc, rep = h.solve(p.z, p.rhs_idx, tol=1e-10, tile=A, zchunk=A, shift_chunk=A,
                          cache_mode=A)
        assert rc == scocg.OK
        return rep, h.green_columns()
    finally:
        h.destroy()


def shape(rep):
    return rep["tile"], rep["zchunk"], rep["shift_chunk"], rep["cache_mode"]


def test_tune_records_persist_across_handles(tmp_path, monkeypatch):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SCOCG_TUNE_CACHE", str(path))
    p = W.tiny_fp64()
    t0 = time.perf_counter()
    r1, G1 = solve_auto(p)
    assert r1["tuned"] and r1["tune_ms"] > 0
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["arch"].startswith("gfx") and rec["precision"] == "fp64"
    assert rec["grid"] == [p.nx, p.ny, p.nz] and rec["nf"] == p.nf
    assert (rec["block_width"], rec["energies"], rec["rows"]) == (8, p.z.size, p.rhs_idx.size)
    assert (rec["tile"], rec["zchunk"], rec["shift_chunk"], rec["cache_mode"]) == shape(r1)
    # a fresh handle (empty in-handle cache) takes the record: no trials, same columns
    r2, G2 = solve_auto(p)
    assert not r2["tuned"] and r2["tune_ms"] == 0 and shape(r2) == shape(r1)
    assert np.array_equal(G1, G2)
    assert len(path.read_text().splitlines()) == 1
    # another shape of the same grid (fewer energies) is a different key: it tunes
    q = p.with_(z=p.z[:8])
    r3, _ = solve_auto(q)
    assert r3["tuned"]
    assert len(path.read_text().splitlines()) == 2
    print(f"tune records: {time.perf_counter() - t0:.1f} s", flush=True)


def test_out_of_range_tune_record_is_ignored(tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SCOCG_TUNE_CACHE", str(path))
    p = W.tiny_fp64()
    r1, _ = solve_auto(p)
    rec = json.loads(path.read_text().splitlines()[0])
    # the same key with an invalid tile and shift chunk, written in the library's form
    bad = path.read_text().splitlines()[0]
    bad = bad.replace(f"\"tile\": {rec['tile']},", "\"tile\": 9,")
    bad = bad.replace(f"\"shift_chunk\": {rec['shift_chunk']},", "\"shift_chunk\": 3,")
    path.write_text(bad + "\n")
    r2, _ = solve_auto(p)
    assert r2["tuned"], "an out-of-range record must not be used"
    assert r2["tile"] in (1, 2, 3, 4) and r2["shift_chunk"] in (1, 4, 16)
    assert len(path.read_text().splitlines()) == 2


def test_recorded_medium_shape_is_taken_by_the_library(tmp_path, monkeypatch):
    """The bench's recorded MI355X shape for the medium workload (the repository's
    tuned_shapes.jsonl) is read by the library itself: an autotuned solve of that
    workload runs no trials and reports exactly the recorded shape."""
    import os
    import shutil
    rec_file = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_1502_00081_amd", "tuned_shapes.jsonl")
    path = tmp_path / "tune.jsonl"
    shutil.copyfile(rec_file, path)
    monkeypatch.setenv("SCOCG_TUNE_CACHE", str(path))
    rec = [json.loads(l) for l in path.read_text().splitlines() if '"grid": [48, 48, 96]' in l][0]
    p = W.medium_fp64()
    h = scocg.create_from_problem(p, precision=scocg.FP64)
    try:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        rc, rep = h.solve(p.z, p.rhs_idx, tol=1e-8, max_iter=18, tile=A, zchunk=A,
                          shift_chunk=A, cache_mode=A, zchunk_mu=A)
    finally:
        h.destroy()
    assert rc in (scocg.OK, scocg.NOT_ALL_CONVERGED)
    if arch != rec["arch"]:
        assert rep["tuned"]  # another architecture has no record and tunes
        return
    assert not rep["tuned"] and rep["tune_ms"] == 0
    assert (rep["tile"], rep["zchunk"], rep["shift_chunk"], rep["cache_mode"],
            rep["zchunk_mu"]) == (rec["tile"], rec["zchunk"], rec["shift_chunk"],
                                  rec["cache_mode"], rec["zchunk_mu"])
    assert len(path.read_text().splitlines()) == 1  # nothing appended
