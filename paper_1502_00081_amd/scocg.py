"""Python binding of the scocg C ABI (include/scocg.h): argument marshalling only.

Every step of the solve runs in the HIP library libscocg.so; this module
converts numpy arrays to pointers and back.  Device buffers may be passed as
torch tensors (their data_ptr() is used); PyTorch is only a source of device
memory and streams here.  If the library has not been built, loading fails
with an error -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscocg.so")

OK, EINVAL, ENOMEM, EHIP, ENOSOLVE = 0, -1, -2, -3, -4
NOT_ALL_CONVERGED, BREAKDOWN = 1, 2
FP64, MIXED = 0, 1
PAIR_CONVERGED, PAIR_MAXITER, PAIR_BREAKDOWN, PAIR_STALLED = 0, 1, 2, 4
C128, C64 = 0, 1

EXPORTS = ("scocg_create", "scocg_solve", "scocg_batch_solve", "scocg_green_columns",
           "scocg_apply_h", "scocg_apply_h_noalloc", "scocg_obm", "scocg_stream_probe",
           "scocg_destroy", "scocg_last_error", "scocg_struct_size")
SCRATCH_BYTES = 64 << 20  # SCOCG_SCRATCH_BYTES: workspace of the allocation-free apply
AUTO = -1  # SCOCG_AUTO: autotuned launch shape


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("nf", C.c_int32), ("n_proj", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("init_seed", C.c_int32),
                ("seed_switch", C.c_int32), ("full", C.c_int32), ("refine", C.c_int32),
                ("poll_every", C.c_int32), ("use_graph", C.c_int32), ("timing", C.c_int32),
                ("tile", C.c_int32), ("zchunk", C.c_int32), ("shift_chunk", C.c_int32),
                ("conventional", C.c_int32), ("aux_seed", C.c_int32),
                ("seed_z", C.c_double * 2), ("symmetric", C.c_int32),
                ("cache_mode", C.c_int32), ("zchunk_mu", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("est_resid", C.c_void_p), ("true_resid", C.c_void_p),
                ("status", C.c_void_p), ("seed_iters", C.c_int64), ("n_switches", C.c_int64),
                ("refined", C.c_int64), ("solve_ms", C.c_double), ("block_iters", C.c_int64),
                ("block_width", C.c_int32), ("n_blocks", C.c_int32),
                ("kernel_ms", C.c_double * 6), ("kernel_launches", C.c_int64 * 6),
                ("tile_used", C.c_int32), ("zchunk_used", C.c_int32),
                ("shift_chunk_used", C.c_int32), ("tuned", C.c_int32), ("tune_ms", C.c_double),
                ("cache_mode_used", C.c_int32), ("zchunk_mu_used", C.c_int32)]

class Problem(C.Structure):
    _fields_ = [("K", C.c_int32), ("z", C.c_void_p), ("R", C.c_int32), ("rhs_idx", C.c_void_p),
                ("nS", C.c_int32), ("s_idx", C.c_void_p)]


KERNEL_FAMILIES = ("proj", "mu", "alpha", "update", "control", "shift")


class ScocgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"scocg error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libscocg.so (built by paper_1502_00081_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -m paper_1502_00081_amd.build)")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.scocg_create.argtypes = [C.POINTER(Grid), P, P, C.c_int32, P, P, P, P, C.c_int32, P,
                                 C.POINTER(P)]
    lib.scocg_create.restype = C.c_int
    lib.scocg_solve.argtypes = [P, C.c_int32, P, C.c_int32, P, C.c_int32, P,
                                C.POINTER(SolveOpts), C.POINTER(Report)]
    lib.scocg_solve.restype = C.c_int
    lib.scocg_green_columns.argtypes = [P, P, C.c_int32, C.c_int32]
    lib.scocg_green_columns.restype = C.c_int
    lib.scocg_apply_h.argtypes = [P, P, P]
    lib.scocg_apply_h.restype = C.c_int
    lib.scocg_apply_h_noalloc.argtypes = [P, P, P]
    lib.scocg_apply_h_noalloc.restype = C.c_int
    lib.scocg_destroy.argtypes = [P]
    lib.scocg_destroy.restype = None
    lib.scocg_last_error.argtypes = []
    lib.scocg_last_error.restype = C.c_char_p
    lib.scocg_struct_size.argtypes = [C.c_int32]
    lib.scocg_struct_size.restype = C.c_int64
    lib.scocg_batch_solve.argtypes = [C.c_int32, P, P, C.POINTER(SolveOpts), P, P]
    lib.scocg_batch_solve.restype = C.c_int
    lib.scocg_obm.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P]
    lib.scocg_obm.restype = C.c_int
    lib.scocg_stream_probe.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int64, C.c_int32, P]
    lib.scocg_stream_probe.restype = C.c_int
    for which, mirror in enumerate((Grid, SolveOpts, Report, Problem)):
        if lib.scocg_struct_size(which) != C.sizeof(mirror):
            raise RuntimeError(f"{path}: {mirror.__name__} is {C.sizeof(mirror)} bytes here, "
                               f"{lib.scocg_struct_size(which)} in the library")
    _lib = lib
    return lib


def last_error() -> str:
    return load().scocg_last_error().decode()


def _check(rc):
    if rc < 0:
        raise ScocgError(rc, last_error())
    return rc


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _stream_ptr(stream):
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream))


def _dev_ptr(t):
    return int(t.data_ptr()) if hasattr(t, "data_ptr") else int(t)


def _opts(tol, max_iter, init_seed, seed_switch, full, refine, poll_every, use_graph, timing,
          tile, zchunk, shift_chunk, conventional=False, seed_z=None, symmetric=False,
          cache_mode=0, zchunk_mu=0):
    o = SolveOpts(float(tol), int(max_iter), int(init_seed), int(bool(seed_switch)),
                  int(bool(full)), int(refine), int(poll_every), int(bool(use_graph)),
                  int(timing), int(tile), int(zchunk), int(shift_chunk),
                  int(bool(conventional)))
    if seed_z is not None:
        o.aux_seed = 1
        o.seed_z[0], o.seed_z[1] = float(np.real(seed_z)), float(np.imag(seed_z))
    o.symmetric = int(bool(symmetric))
    o.cache_mode = int(cache_mode)
    o.zchunk_mu = int(zchunk_mu)
    return o


def _new_report(K, R):
    arrays = dict(iters=np.zeros((K, R), np.int64), est=np.zeros((K, R)),
                  true_resid=np.zeros((K, R)), status=np.zeros((K, R), np.int32))
    rep = Report()
    rep.iters, rep.est_resid = arrays["iters"].ctypes.data, arrays["est"].ctypes.data
    rep.true_resid, rep.status = arrays["true_resid"].ctypes.data, arrays["status"].ctypes.data
    return rep, arrays


def _report_dict(rep, arrays):
    return dict(arrays, seed_iters=rep.seed_iters, n_switches=rep.n_switches,
                refined=rep.refined, solve_ms=rep.solve_ms, block_iters=rep.block_iters,
                block_width=rep.block_width, n_blocks=rep.n_blocks,
                kernel_ms=dict(zip(KERNEL_FAMILIES, list(rep.kernel_ms))),
                kernel_launches=dict(zip(KERNEL_FAMILIES, list(rep.kernel_launches))),
                tile=rep.tile_used, zchunk=rep.zchunk_used, shift_chunk=rep.shift_chunk_used,
                tuned=bool(rep.tuned), tune_ms=rep.tune_ms, cache_mode=rep.cache_mode_used,
                zchunk_mu=rep.zchunk_mu_used)


class Handle:
    """One uploaded Hamiltonian (scocg_create) and its last solve."""

    def __init__(self, ptr, n, keep):
        self._h = C.c_void_p(ptr)
        self.n = n
        self._keep = keep
        self.last = None

    def solve(self, z, rhs_idx, s_idx=None, tol=1e-10, max_iter=100000, init_seed=-1,
              seed_switch=True, full=False, refine=0, poll_every=0, use_graph=False, timing=0,
              tile=0, zchunk=0, shift_chunk=0, conventional=False, seed_z=None,
              symmetric=False, cache_mode=0, zchunk_mu=0):
        """scocg_solve; returns (rc, report dict with [K, R] arrays).  conventional=True runs
        every (energy, column) pair as its own recurrence (the comparison sweep).  seed_z (a
        complex energy, not necessarily one of z) starts the seed recurrence there.
        symmetric=True (S = the RHS set) keeps each block's rows from its first column on
        and mirrors the rest."""
        lib = load()
        z = _c(z, np.complex128)
        rhs = _c(rhs_idx, np.int64)
        sp = None if s_idx is None else _c(s_idx, np.int64)
        o = _opts(tol, max_iter, init_seed, seed_switch, full, refine, poll_every, use_graph,
                  timing, tile, zchunk, shift_chunk, conventional, seed_z, symmetric, cache_mode,
                  zchunk_mu)
        rep, arrays = _new_report(z.size, rhs.size)
        rc = lib.scocg_solve(self._h, z.size, z.ctypes.data, rhs.size, rhs.ctypes.data,
                             0 if sp is None else sp.size,
                             None if sp is None else sp.ctypes.data, C.byref(o), C.byref(rep))
        _check(rc)
        nrows = self.n if full else (sp.size if sp is not None else rhs.size)
        self.last = (z.size, rhs.size, nrows)
        return rc, _report_dict(rep, arrays)

    def green_columns(self, out=None, dtype=C128):
        """scocg_green_columns into `out` (torch device tensor or numpy array), or a new
        numpy array [K, R, nS]."""
        lib = load()
        if out is None:
            K, R, nS = self.last
            out = np.zeros((K, R, nS), np.complex128 if dtype == C128 else np.complex64)
        if isinstance(out, np.ndarray):
            assert out.flags.c_contiguous
            _check(lib.scocg_green_columns(self._h, out.ctypes.data, dtype, 0))
        else:
            _check(lib.scocg_green_columns(self._h, _dev_ptr(out), dtype, 1))
        return out

    def apply_h(self, x_dev, y_dev):
        """scocg_apply_h on complex128 device vectors (torch tensors or raw pointers)."""
        _check(load().scocg_apply_h(self._h, _dev_ptr(x_dev), _dev_ptr(y_dev)))

    def apply_h_noalloc(self, x_dev, y_dev):
        """scocg_apply_h_noalloc: the same apply with no device allocation (workspace in
        the library's per-GPU scratch array)."""
        _check(load().scocg_apply_h_noalloc(self._h, _dev_ptr(x_dev), _dev_ptr(y_dev)))

    def obm(self, K, M, L, g_dev, sig_l_dev, sig_r_dev, gt_dev=None, phase_ms=None):
        """scocg_obm on device buffers (torch tensors or raw pointers), all complex128 and
        column-major per energy.  Returns (rc, T [K] complex, dos [K]); phase_ms (a float64
        array of 4) receives the device time per phase when given."""
        trans = np.zeros(K, np.complex128)
        dos = np.zeros(K, np.float64)
        if phase_ms is not None:
            assert phase_ms.dtype == np.float64 and phase_ms.size >= 4
        rc = load().scocg_obm(self._h, K, M, L, _dev_ptr(g_dev), _dev_ptr(sig_l_dev),
                              _dev_ptr(sig_r_dev), None if gt_dev is None else _dev_ptr(gt_dev),
                              trans.ctypes.data, dos.ctypes.data,
                              None if phase_ms is None else phase_ms.ctypes.data)
        _check(rc)
        return rc, trans, dos

    def stream_probe(self, buf_dev, nbytes, mode, nontemporal=True, reps=10):
        """scocg_stream_probe on a device buffer of nbytes: GB/s of the pass-like access mix
        (mode 0 copy, 1 two reads + one write, 2 reads only)."""
        g = np.zeros(1)
        _check(load().scocg_stream_probe(self._h, int(mode), int(bool(nontemporal)),
                                         _dev_ptr(buf_dev), int(nbytes), int(reps),
                                         g.ctypes.data))
        return float(g[0])

    def destroy(self):
        if self._h:
            load().scocg_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def create(nx, ny, nz, nf, coef, vloc, atom_ptr=None, atom_idx=None, atom_P=None, atom_D=None,
           precision=FP64, stream=None) -> Handle:
    """scocg_create from numpy arrays (shapes as in include/scocg.h)."""
    lib = load()
    coef = _c(coef, np.float64)
    vloc = _c(vloc, np.float64)
    n_atoms = 0 if atom_ptr is None else int(np.asarray(atom_ptr).size - 1)
    keep = [coef, vloc]
    ptrs = [None, None, None, None]
    n_proj = 0
    if n_atoms > 0:
        ap, ai = _c(atom_ptr, np.int64), _c(atom_idx, np.int64)
        aP, aD = _c(atom_P, np.float64), _c(atom_D, np.float64)
        n_proj = aD.shape[1]
        keep += [ap, ai, aP, aD]
        ptrs = [a.ctypes.data for a in (ap, ai, aP, aD)]
    g = Grid(nx, ny, nz, nf, n_proj)
    out = C.c_void_p()
    _check(lib.scocg_create(C.byref(g), coef.ctypes.data, vloc.ctypes.data, n_atoms, *ptrs,
                            int(precision), _stream_ptr(stream), C.byref(out)))
    return Handle(out.value, nx * ny * nz, keep)


def create_from_problem(p, precision=FP64, stream=None) -> Handle:
    """scocg_create for an object with the fields of workload.Problem."""
    return create(p.nx, p.ny, p.nz, p.nf, p.coef, p.vloc, p.atom_ptr, p.atom_idx, p.atom_P,
                  p.atom_D, precision=precision, stream=stream)


def batch_solve(handles, problems, tol=1e-10, max_iter=100000, seed_switch=True, full=False,
                refine=0, poll_every=0, use_graph=False, timing=0, tile=0, zchunk=0,
                shift_chunk=0, symmetric=False, cache_mode=0, zchunk_mu=0):
    """scocg_batch_solve over regions; problems: [(z, rhs_idx) or (z, rhs_idx, s_idx)].
    Returns (rc, [report dict per region], region_ms [n])."""
    lib = load()
    n = len(handles)
    assert len(problems) == n
    keep, probs, reps, arrays = [], (Problem * n)(), (Report * n)(), []
    for i, pr in enumerate(problems):
        z = _c(pr[0], np.complex128)
        rhs = _c(pr[1], np.int64)
        sp = _c(pr[2], np.int64) if len(pr) > 2 and pr[2] is not None else None
        keep += [z, rhs, sp]
        probs[i] = Problem(z.size, z.ctypes.data, rhs.size, rhs.ctypes.data,
                           0 if sp is None else sp.size, None if sp is None else sp.ctypes.data)
        rep, arr = _new_report(z.size, rhs.size)
        reps[i] = rep
        arrays.append(arr)
        nrows = handles[i].n if full else (sp.size if sp is not None else rhs.size)
        handles[i].last = (z.size, rhs.size, nrows)
    hs = (C.c_void_p * n)(*[h._h.value for h in handles])
    o = _opts(tol, max_iter, -1, seed_switch, full, refine, poll_every, use_graph, timing, tile,
              zchunk, shift_chunk, symmetric=symmetric, cache_mode=cache_mode,
              zchunk_mu=zchunk_mu)
    region_ms = np.zeros(n)
    rc = lib.scocg_batch_solve(n, hs, probs, C.byref(o), reps, region_ms.ctypes.data)
    _check(rc)
    return rc, [_report_dict(reps[i], arrays[i]) for i in range(n)], region_ms


def open_boundary(handle, z, idx, M, L, sig_l, sig_r, tol=1e-10, max_iter=100000, device=None,
                  **solve_kw):
    """Unperturbed columns on idx (scocg_solve, symmetric rows by default), then the
    matching (scocg_obm).

    idx = (left block, right block, extra rows) grid indices; sig_l, sig_r [K, M, M]
    complex (matrix orientation).  Returns a dict with the solve's rc and report, the
    matching's rc, T [K] complex, dos [K] and gt [K, D, D] (numpy, matrix orientation:
    gt[k][r, c] = G_T(Z_k)[idx_r, idx_c])."""
    import torch

    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    z = np.atleast_1d(np.asarray(z, np.complex128))
    idx = np.asarray(idx, np.int64)
    K, D = z.size, idx.size
    assert D == 2 * M + L
    solve_kw.setdefault("symmetric", True)
    rc, rep = handle.solve(z, idx, tol=tol, max_iter=max_iter, **solve_kw)
    g = torch.empty((K, D, D), dtype=torch.complex128, device=dev)
    handle.green_columns(out=g)
    # column-major per energy: element (r, c) at r + M c, i.e. the transposed matrix
    sl = torch.from_numpy(np.ascontiguousarray(np.transpose(sig_l, (0, 2, 1)))).to(dev)
    sr = torch.from_numpy(np.ascontiguousarray(np.transpose(sig_r, (0, 2, 1)))).to(dev)
    gt = torch.empty_like(g)
    torch.cuda.synchronize(dev)
    rc_obm, T, dos = handle.obm(K, M, L, g, sl, sr, gt)
    return {"rc": rc, "report": rep, "rc_obm": rc_obm, "T": T, "dos": dos,
            "gt": gt.cpu().numpy().transpose(0, 2, 1), "g": g.cpu().numpy().transpose(0, 2, 1)}
