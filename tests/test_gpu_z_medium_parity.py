"""Full-size parity on the medium workload (48x48x96 grid, 40 atoms with projectors,
128 energies in [-0.6, 0.6] Ha, eta = 1e-3, 32 + 32 boundary columns), including the
top of the energy window, where the slowest pairs and every seed switch are.

Three solves through the C ABI:
  * the benchmarked launch (projected storage, every energy and column, tol 1e-8):
    size-independent properties on every pair and the rows of the sampled pairs;
  * full storage, 5 energies (0, 40, 96, 120, 127) x 8 columns (4 on each boundary
    plane), tol 1e-8: every pair's true residual ||e_j - (z_k - H) x||, evaluated with
    the oracle's operator, within 1.1 tol;
  * the same pairs at tol 1e-12: six of them -- both planes, two at the top of the
    window, one in the middle, the bottom -- against the oracle's conventional COCG at
    tol 1e-13 on every row, within 1e-10 relative per column.
The oracle pairs need up to about 2e4 iterations of a 221184-point operator; they run
in two groups (bottom and middle of the window, then the top), each one call of the
oracle's OpenMP loop over its pairs.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1502_00081_amd import scocg
from paper_1502_00081_amd import workload as W

torch = pytest.importorskip("torch")

ENERGIES = np.array([0, 40, 96, 120, 127])
COLS = np.array([0, 1, 2, 3, 32, 33, 34, 35])  # 4 on iz = 0, 4 on iz = nz - 1
# (index into ENERGIES, index into COLS): both planes at the top, plane 1 near the top,
# the middle and the bottom of the window
ORACLE_PAIRS = [(4, 0), (4, 7), (3, 2), (3, 5), (2, 4), (0, 1)]
ORACLE_TOL = 1e-13


def say(msg):
    line = f"[{time.strftime('%H:%M:%S')}] {msg}\n"
    path = os.environ.get("SCOCG_TEST_PROGRESS")
    if path:
        with open(path, "a") as f:
            f.write(line)
    sys.__stderr__.write(line)
    sys.__stderr__.flush()


def subproblem():
    p = W.medium_fp64()
    return p, p.with_(z=p.z[ENERGIES], rhs_idx=p.rhs_idx[COLS])


def true_residuals(p, G):
    K, R, _ = G.shape
    out = np.zeros((K, R))
    for k in range(K):
        for j in range(R):
            t = -(p.z[k] * G[k, j] - oracle.apply_h(p, G[k, j]))
            t[p.rhs_idx[j]] += 1.0
            out[k, j] = np.linalg.norm(t)
    return out


@pytest.mark.gpu
@pytest.mark.timeout(900)
def test_medium_full_size_parity_including_top_of_window():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    base, q = subproblem()
    eta = base.z.imag.min()
    # 1. the benchmarked launch: every energy and column, projected storage, tol 1e-8
    h = scocg.create_from_problem(base, precision=scocg.FP64)
    try:
        t0 = time.perf_counter()
        rc, rep = h.solve(base.z, base.rhs_idx, tol=1e-8, use_graph=True, max_iter=40000)
        say(f"medium projected: rc={rc}, {rep['seed_iters']} seed iterations, "
            f"{rep['n_switches']} switches, {time.perf_counter() - t0:.1f} s")
        assert rc == scocg.OK and (rep["status"] == scocg.PAIR_CONVERGED).all()
        Gp = h.green_columns()  # [K, R, R]
    finally:
        h.destroy()
    for k in range(0, base.z.size, 9):
        g = Gp[k].T  # g[i, j] = G(S_i, rhs_j)
        assert np.abs(g - g.T).max() <= 2e-8 / eta
        assert (np.diag(g).imag < 0).all()
    assert np.abs(Gp).max() <= 1.0 / eta
    # 2. full storage on the subsample: tol 1e-8 (true residuals) and tol 1e-12
    h = scocg.create_from_problem(q, precision=scocg.FP64)
    try:
        t0 = time.perf_counter()
        rc8, rep8 = h.solve(q.z, q.rhs_idx, tol=1e-8, full=True, use_graph=True, max_iter=40000)
        G8 = h.green_columns()  # [5, 8, N]
        say(f"medium subsample tol 1e-8 full storage: rc={rc8}, {rep8['seed_iters']} seed "
            f"iterations, {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        rc12, rep12 = h.solve(q.z, q.rhs_idx, tol=1e-12, full=True, use_graph=True,
                              max_iter=60000)
        G12 = h.green_columns()
        say(f"medium subsample tol 1e-12 full storage: rc={rc12}, {rep12['seed_iters']} seed "
            f"iterations, {time.perf_counter() - t0:.1f} s")
    finally:
        h.destroy()
    assert rc8 == scocg.OK and rc12 == scocg.OK
    assert (rep8["status"] == scocg.PAIR_CONVERGED).all()
    assert (rep12["status"] == scocg.PAIR_CONVERGED).all()
    tr = true_residuals(q, G8)
    say(f"true residuals at tol 1e-8 (oracle operator): max {tr.max():.3e}, "
        f"median {np.median(tr):.3e}")
    assert (tr <= 1.1e-8).all(), tr.max()
    # the library's own FP64 residual pass agrees with the oracle's operator
    np.testing.assert_allclose(rep8["true_resid"], tr, rtol=1e-6, atol=1e-15)
    tr12 = true_residuals(q, G12)
    say(f"true residuals at tol 1e-12: max {tr12.max():.3e}, median {np.median(tr12):.3e}")
    # the projected rows of the benchmarked launch are those columns on S, within the
    # resolvent bound of the two residuals
    for a, k in enumerate(ENERGIES):
        for b, j in enumerate(COLS):
            d = np.linalg.norm(Gp[k, j] - G12[a, b, base.rhs_idx])
            assert d <= (1.1e-8 + tr12[a, b]) / eta, (k, j, d)
    # 3. the oracle's columns: the lower pairs, then the top of the window
    for group in ([pq for pq in ORACLE_PAIRS if ENERGIES[pq[0]] < 120],
                  [pq for pq in ORACLE_PAIRS if ENERGIES[pq[0]] >= 120]):
        t0 = time.perf_counter()
        ref, it, st, _ = oracle.cocg_unit_columns(q, q.z, q.rhs_idx, np.arange(q.n), group,
                                                  tol=ORACLE_TOL, max_iter=200000)
        say(f"oracle: {len(group)} pairs at tol {ORACLE_TOL:g}, iterations {list(map(int, it))}, "
            f"{time.perf_counter() - t0:.0f} s")
        assert (st == oracle.CONVERGED).all(), st
        for s, (a, b) in enumerate(group):
            d = np.linalg.norm(G12[a, b] - ref[s])
            rel = d / np.linalg.norm(ref[s])
            say(f"pair (k={ENERGIES[a]}, column {COLS[b]}): rel {rel:.3e}, GPU iterations "
                f"{rep12['iters'][a, b]}, oracle {it[s]}")
            assert rel <= 1e-10, (ENERGIES[a], COLS[b], rel)
