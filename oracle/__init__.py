"""CPU FP64 oracle: plain, slow, independent reference for the Green's-function columns.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's CPU
baseline leg may import this package.  It shares no code with the GPU library
and never imports it; its inputs are plain arrays (any object with the fields
nx, ny, nz, nf, coef, vloc, atom_ptr, atom_idx, atom_P, atom_D).

Functions (each a thin ctypes marshaller over oracle.c):
  apply_h(op, x)                     y = H x                           (Sec. 2A, Eq. 2)
  cocg(op, z, b, ...)                conventional COCG, one system       (App., Eqs. A1-A6)
  cocg_unit_columns(op, pairs, ...)  many (z_k, e_j) systems, OpenMP     (Sec. 3B, Eq. 17)
  shifted_cocg(op, z, b, ...)        shifted COCG + seed switching       (App., Eqs. A7-A13)
The submodule oracle.obm holds the open-boundary reference: perturbed Green's
function blocks by direct inversion of Eq. 13, the Fisher-Lee transmission
(Eq. 14) and the density of states.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def compile_source(src: str, out: str) -> str:
    """gcc -O2 (OpenMP, no fast-math) of one oracle C source into a shared library."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


class _Op(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("nf", C.c_int32), ("n_proj", C.c_int32),
                ("coef", C.c_void_p), ("vloc", C.c_void_p),
                ("n_atoms", C.c_int32), ("atom_ptr", C.c_void_p), ("atom_idx", C.c_void_p),
                ("atom_P", C.c_void_p), ("atom_D", C.c_void_p)]


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = C.c_void_p
    lib.oracle_apply_h.argtypes = [P, P, P]
    lib.oracle_apply_h.restype = None
    lib.oracle_cocg.argtypes = [P, P, P, C.c_double, C.c_int64, P, P,
                                P, P, P, P, P, C.c_int64, P]
    lib.oracle_cocg.restype = C.c_int
    lib.oracle_cocg_unit_batch.argtypes = [P, C.c_int64, P, P, P, C.c_int64, C.c_double,
                                           C.c_int64, P, P, P, P]
    lib.oracle_cocg_unit_batch.restype = C.c_int
    lib.oracle_shifted_cocg.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_double,
                                        C.c_int64, P, P, P, P, P, P]
    lib.oracle_shifted_cocg.restype = C.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(C.CDLL(_LIB))
    return _lib


class _OpHolder:
    """Keeps contiguous copies of the operator arrays alive with the struct."""

    def __init__(self, p):
        self.coef = np.ascontiguousarray(p.coef, dtype=np.float64)
        self.vloc = np.ascontiguousarray(p.vloc, dtype=np.float64)
        self.ptr = np.ascontiguousarray(p.atom_ptr, dtype=np.int64)
        self.idx = np.ascontiguousarray(p.atom_idx, dtype=np.int64)
        self.P = np.ascontiguousarray(p.atom_P, dtype=np.float64)
        self.D = np.ascontiguousarray(p.atom_D, dtype=np.float64)
        n_proj = self.P.shape[1] if self.P.ndim == 2 and self.P.shape[0] else (
            self.D.shape[1] if self.D.ndim == 2 else 0)
        assert self.coef.shape == (3, p.nf + 1)
        assert self.vloc.shape == (p.nx * p.ny * p.nz,)
        self.s = _Op(p.nx, p.ny, p.nz, p.nf, n_proj, self.coef.ctypes.data,
                     self.vloc.ctypes.data, self.ptr.shape[0] - 1, self.ptr.ctypes.data,
                     self.idx.ctypes.data, self.P.ctypes.data, self.D.ctypes.data)
        self.n = p.nx * p.ny * p.nz

    @property
    def ref(self):
        return C.byref(self.s)


def _cz(z):
    return np.array([z], dtype=np.complex128)


def _ptr(a):
    return None if a is None else a.ctypes.data


def apply_h(p, x):
    """y = H x for complex x of length N (Sec. 2A, Eq. 2; nonlocal blocks as P D P^T)."""
    op = _OpHolder(p)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().oracle_apply_h(op.ref, x.ctypes.data, y.ctypes.data)
    return y


def cocg(p, z, b, tol=1e-12, max_iter=100000, history=False, snap_iter=-1):
    """Conventional COCG on (z - H) x = b (App., Eqs. A1-A6).

    Returns dict(x, iters, status, alpha, beta, res, snap)."""
    lib = _load()
    op = _OpHolder(p)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.empty(op.n, np.complex128)
    it = np.zeros(1, np.int64)
    h = [np.zeros(max_iter) for _ in range(5)] if history else [None] * 5
    snap = np.zeros(op.n, np.complex128) if snap_iter >= 0 else None
    zz = _cz(z)
    st = lib.oracle_cocg(op.ref, zz.ctypes.data, b.ctypes.data, tol, max_iter, x.ctypes.data,
                         it.ctypes.data, *[_ptr(a) for a in h], snap_iter, _ptr(snap))
    n = int(it[0])
    out = dict(x=x, iters=n, status=st, snap=snap)
    if history:
        out["alpha"] = h[0][:n] + 1j * h[1][:n]
        out["beta"] = h[2][:n] + 1j * h[3][:n]
        out["res"] = h[4][:n]
    return out


def cocg_unit_columns(p, z, rhs, rows, pairs, tol=1e-12, max_iter=100000, full=False):
    """Independent conventional COCG for each (k, j) in `pairs` on (z_k - H) x = e_{rhs[j]}.

    Returns (G [n_pairs, n_rows], iters [n_pairs], status [n_pairs], x_full or None)."""
    lib = _load()
    op = _OpHolder(p)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    zs = np.ascontiguousarray(np.asarray(z, np.complex128)[pairs[:, 0]])
    rr = np.ascontiguousarray(np.asarray(rhs, np.int64)[pairs[:, 1]])
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    ns = pairs.shape[0]
    out = np.zeros((ns, rows.size), np.complex128)
    iters = np.zeros(ns, np.int64)
    status = np.zeros(ns, np.int32)
    xf = np.zeros((ns, op.n), np.complex128) if full else None
    rc = lib.oracle_cocg_unit_batch(op.ref, ns, zs.ctypes.data, rr.ctypes.data, rows.ctypes.data,
                                    rows.size, tol, max_iter, out.ctypes.data, iters.ctypes.data,
                                    status.ctypes.data, _ptr(xf))
    if rc != 0:
        raise MemoryError("oracle_cocg_unit_batch: allocation failed")
    return out, iters, status, xf


def shifted_cocg(p, z, b, seed0, seed_switch=True, tol=1e-10, max_iter=100000):
    """Shifted COCG with collinear residuals and seed switching (App., Eqs. A7-A13).

    Returns dict(x [K, N], iters, status, est, n_switch, seed_final)."""
    lib = _load()
    op = _OpHolder(p)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    K = z.size
    x = np.zeros((K, op.n), np.complex128)
    iters = np.zeros(K, np.int64)
    status = np.zeros(K, np.int32)
    est = np.zeros(K)
    nsw = np.zeros(1, np.int32)
    sf = np.zeros(1, np.int32)
    lib.oracle_shifted_cocg(op.ref, K, z.ctypes.data, b.ctypes.data, int(seed0), int(bool(seed_switch)),
                            tol, max_iter, x.ctypes.data, iters.ctypes.data, status.ctypes.data,
                            est.ctypes.data, nsw.ctypes.data, sf.ctypes.data)
    return dict(x=x, iters=iters, status=status, est=est, n_switch=int(nsw[0]),
                seed_final=int(sf[0]))


CONVERGED, MAXITER, BREAKDOWN = 0, 1, 2
