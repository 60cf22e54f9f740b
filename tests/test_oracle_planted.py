"""The oracle's pins have teeth: plant a plausible mistake in a copy of the
oracle source (on the CPU), rebuild it, and check that a pin catches it.

Each mutation is a one-line textual edit of oracle.c; the copy is compiled
into a temporary directory and bound in place of the real oracle for the
duration of one check.
"""
import ctypes as C
import os

import numpy as np
import pytest

import oracle
from paper_1502_00081_amd import workload as W
from tests import dense_ref as D

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = {
    # the COCG bilinear form conjugated (a Hermitian inner product)
    "conjugated_form": ("s += u[i] * v[i];", "s += conj(u[i]) * v[i];"),
    # z truncation lost: periodic in z as well
    "periodic_z": ("if (iz + k >= 0 && iz + k < nz)\n                        acc += op->coef[2 * (nf + 1) + ak] * x[ix + nx * (iy + ny * (iz + k))];",
                   "acc += op->coef[2 * (nf + 1) + ak] * x[ix + nx * (iy + ny * wrap(iz + k, nz))];"),
    # projector block applied with the transposed D index (channel of another atom)
    "projector_d_index": ("c[l] *= op->atom_D[a * np + l];", "c[l] *= op->atom_D[l * np + a % np];"),
    # sign of sigma in the pi recurrence (Eq. A8)
    "sigma_sign": ("(1.0 + c + alpha * sigma) * pi[k]", "(1.0 + c - alpha * sigma) * pi[k]"),
    # the three-term recurrence's last term dropped (Eq. A3)
    "drop_r_prev": ("r_next[i] = (1.0 + c) * r[i] - alpha * ar[i] - c * r_prev[i];\n        const cplx rho_next",
                    "r_next[i] = (1.0 + c) * r[i] - alpha * ar[i];\n        const cplx rho_next"),
    # seed switching rebases pi with the wrong index (n+1 factor for both)
    "switch_rebase": ("pi[k] /= f_cur;", "pi[k] /= f_next;"),
    # the shift's x takes the new direction p_{n+1} instead of p_n (Eqs. A11-A12 order)
    "x_uses_new_p": ("x_out[k * n + i] += ak * p[k * n + i];\n                p[k * n + i] = r_next[i] / pi_next[k] + bk * p[k * n + i];",
                     "p[k * n + i] = r_next[i] / pi_next[k] + bk * p[k * n + i];\n                x_out[k * n + i] += ak * p[k * n + i];"),
}


@pytest.fixture
def mutated(tmp_path, monkeypatch):
    def make(name):
        old, new = MUTATIONS[name]
        text = open(SRC).read()
        assert text.count(old) >= 1, name
        src = tmp_path / f"{name}.c"
        src.write_text(text.replace(old, new))
        lib = oracle._bind(C.CDLL(oracle.compile_source(str(src), str(tmp_path / f"{name}.so"))))
        monkeypatch.setattr(oracle, "_lib", lib)
    return make


def _problem(projectors=True):
    return W.make_problem("m", 8, 8, 12, 0.4, 4, 3, projectors, 7, 1e-3, -0.5, 0.5, 3, 3, 7)


def _pin_apply_h():
    p = _problem()
    v = np.random.default_rng(3).standard_normal(p.n) + 0.5j
    y = oracle.apply_h(p, v)
    H = D.dense_h(p)
    return np.abs(y - H @ v).max() <= 1e-12 * np.abs(H @ v).max()


def _pin_cocg_dense():
    p = _problem()
    H = D.dense_h(p)
    b = np.zeros(p.n, complex)
    b[p.rhs_idx[0]] = 1
    ok = True
    for k in (0, 3, 6):
        ref = np.linalg.solve(p.z[k] * np.eye(p.n) - H, b)
        x = oracle.cocg(p, p.z[k], b, tol=1e-12, max_iter=3000)["x"]
        ok &= np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    return ok


def _pin_shifted_dense():
    """Shifted solutions vs dense solves; the energy set puts the seed below the
    spectrum so that it converges early and a seed switch happens mid-run."""
    p = _problem()
    H = D.dense_h(p)
    b = np.zeros(p.n, complex)
    b[p.rhs_idx[1]] = 1
    z = np.array([-4.0, -0.3, 0.2, 0.9, 1.7]) + 1e-3j
    r = oracle.shifted_cocg(p, z, b, seed0=0, tol=1e-11, max_iter=3000)
    ok = r["n_switch"] >= 1
    for k in range(z.size):
        ref = np.linalg.solve(z[k] * np.eye(p.n) - H, b)
        ok &= np.linalg.norm(r["x"][k] - ref) <= 1e-8 * np.linalg.norm(ref)
    return ok


def _pin_collinear():
    """Eq. A7 with pi from Eq. A8 between independent conventional runs."""
    p = _problem()
    b = np.zeros(p.n, complex)
    b[p.rhs_idx[0]] = 1
    n = 20
    seed = oracle.cocg(p, p.z[2], b, tol=0.0, max_iter=n, history=True, snap_iter=n)
    other = oracle.cocg(p, p.z[5], b, tol=0.0, max_iter=n, snap_iter=n)
    sigma = p.z[5] - p.z[2]
    pi_prev, pi, a_prev, b_prev = 1 + 0j, 1 + 0j, 1 + 0j, 0j
    for m in range(n):
        c = b_prev * seed["alpha"][m] / a_prev
        pi_prev, pi = pi, (1 + c + seed["alpha"][m] * sigma) * pi - c * pi_prev
        a_prev, b_prev = seed["alpha"][m], seed["beta"][m]
    rk = other["snap"]
    return np.linalg.norm(rk - seed["snap"] / pi) <= 1e-7 * np.linalg.norm(rk)


def _pin_truncated():
    """After m seed iterations every shift's x equals the conventional COCG iterate at
    its energy (same Krylov iterates, Eqs. A7-A12)."""
    p = _problem()
    b = np.zeros(p.n, complex)
    b[p.rhs_idx[0]] = 1
    m = 12
    s = oracle.shifted_cocg(p, p.z, b, seed0=3, tol=0.0, max_iter=m)
    ok = True
    for k in (0, 5):
        c = oracle.cocg(p, p.z[k], b, tol=0.0, max_iter=m)["x"]
        ok &= np.linalg.norm(s["x"][k] - c) <= 1e-10 * np.linalg.norm(c)
    return ok


def test_pins_pass_on_the_real_oracle():
    assert _pin_apply_h() and _pin_cocg_dense() and _pin_shifted_dense() and _pin_collinear()
    assert _pin_truncated()


@pytest.mark.parametrize("name,pin", [
    # a conjugated form still converges (any consistent Krylov recurrence drives
    # r = b - A x to zero, for the seed and, through pi, for the shifts), so only
    # the collinearity theorem between independent runs exposes it
    ("conjugated_form", _pin_collinear),
    ("periodic_z", _pin_apply_h),
    ("projector_d_index", _pin_apply_h),
    ("sigma_sign", _pin_shifted_dense),
    ("drop_r_prev", _pin_cocg_dense),
    ("switch_rebase", _pin_shifted_dense),
    ("x_uses_new_p", _pin_truncated),
])
def test_planted_mistake_is_caught(mutated, name, pin):
    mutated(name)
    with np.errstate(all="ignore"):
        assert not pin(), f"pin did not catch planted mistake {name}"
