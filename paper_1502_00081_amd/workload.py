"""Seeded synthetic inputs for the unperturbed Green's-function solve.

This module builds inputs only: the real-space grid, the finite-difference
coefficient table of the kinetic operator, a local potential, Kleinman-Bylander
projector blocks, the complex energies and the right-hand-side / output row
sets.  It holds none of the solver's arithmetic.  Both the GPU library's tests
and benchmark and the CPU oracle's tests draw their inputs from here.

Physical setting (Sec. 2A, Eqs. 1-4): a transition region of nx*ny*nz grid
points with spacing h (bohr), periodic in x and y and truncated in z (the
finite T block of the block-tridiagonal Hamiltonian, i.e. zero wavefunction
outside planes 0..nz-1).  Grid index i = ix + nx*(iy + ny*iz), so one x-y plane
(the plane vector Psi(z_k) of Eq. 2) is a contiguous run of nx*ny entries.

The paper's transport workloads use Kohn-Sham potentials of real structures
(a Na wire in Sec. 3C, a C60@(10,10) CNT peapod in Sec. 4).  Those are not
available, so every workload here is synthetic: attractive Gaussian local
potentials and Gaussian-radial s/p projectors, with shapes and sizes that
stand in for the paper's grids.  Units are Hartree and bohr.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import List, Optional

import numpy as np

# Central-difference weights of d^2/dx^2 on a uniform grid, half-width nf
# (weights C_0..C_nf, symmetric).  Standard table (exact for polynomials of
# degree 2*nf+1); the tests check that property independently.
FD_SECOND_DERIVATIVE = {
    1: (Fraction(-2), Fraction(1)),
    2: (Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)),
    3: (Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20), Fraction(1, 90)),
    4: (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315),
        Fraction(-1, 560)),
}

GAUSS_WIDTH = 1.0        # local-potential Gaussian width w (bohr)
PROJ_WIDTH = 0.5         # projector radial Gaussian width (bohr)
PROJ_CUTOFF = 1.6        # projector support radius (bohr)
N_PROJ = 4               # s, p_x, p_y, p_z


@dataclasses.dataclass
class Problem:
    """One transition-region Hamiltonian plus one solve request.

    coef     [3, nf+1] float64: H_kin coefficients along x, y, z in Ha, i.e.
             (H_kin psi)_i = sum_axis sum_{k=-nf..nf} coef[axis,|k|] psi_{i+k e_axis}
    vloc     [N] float64 local potential (Ha)
    atom_ptr [n_atoms+1] int64 CSR offsets into atom_idx / atom_P
    atom_idx [n_entries] int64 grid index of each projector entry
    atom_P   [n_entries, N_PROJ] float64 unit-2-norm projector columns u = h^1.5 p
    atom_D   [n_atoms, N_PROJ] float64 KB energies D_l (Ha)
    z        [K] complex128 energies z_k = E_k + i*eta
    rhs_idx  [R] int64 grid index j of each right-hand side e_j
    s_idx    [nS] int64 output rows (None: the RHS set)
    """
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    nf: int
    coef: np.ndarray
    vloc: np.ndarray
    atom_ptr: np.ndarray
    atom_idx: np.ndarray
    atom_P: np.ndarray
    atom_D: np.ndarray
    z: np.ndarray
    rhs_idx: np.ndarray
    s_idx: Optional[np.ndarray]
    tol: float
    centres: np.ndarray = None  # [n_centres, 3] Gaussian centres (bohr), for reference

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_atoms(self) -> int:
        return int(self.atom_ptr.shape[0] - 1)

    @property
    def rows(self) -> np.ndarray:
        return self.rhs_idx if self.s_idx is None else self.s_idx

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def kinetic_coefficients(h, nf: int) -> np.ndarray:
    """[3, nf+1] coefficients of H_kin = -1/2 Laplacian, per axis.

    h is a scalar or a (hx, hy, hz) triple."""
    hs = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    c = np.array([float(v) for v in FD_SECOND_DERIVATIVE[nf]])
    return np.stack([-0.5 * c / (hh * hh) for hh in hs])


def grid_coords(nx, ny, nz, h):
    """Cartesian coordinates (bohr) of grid points, index order i = ix+nx*(iy+ny*iz)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ix.ravel() * h, iy.ravel() * h, iz.ravel() * h


def _min_image(d, L):
    return d - L * np.round(d / L)


def gaussian_vloc(nx, ny, nz, h, centres, depths, width=GAUSS_WIDTH):
    """V(r) = -sum_a D_a exp(-d^2/(2 w^2)); minimum image in x, y, plain d in z."""
    x, y, zc = grid_coords(nx, ny, nz, h)
    Lx, Ly = nx * h, ny * h
    v = np.zeros(nx * ny * nz)
    for (cx, cy, cz), d in zip(centres, depths):
        dx = _min_image(x - cx, Lx)
        dy = _min_image(y - cy, Ly)
        dz = zc - cz
        v -= d * np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * width * width))
    return v


def kb_projectors(nx, ny, nz, h, centres, rng, width=PROJ_WIDTH, cutoff=PROJ_CUTOFF):
    """Gaussian-radial s and p projectors on points within `cutoff` of each centre.

    Returns atom_ptr, atom_idx, atom_P (unit 2-norm columns), atom_D with
    D_s, D_p ~ U[-1, 1] (D_p shared by the three p channels)."""
    Lx, Ly = nx * h, ny * h
    ptr = [0]
    idx_all: List[np.ndarray] = []
    p_all: List[np.ndarray] = []
    dvals = []
    r = int(np.ceil(cutoff / h)) + 1
    for (cx, cy, cz) in centres:
        bx = np.arange(int(np.floor(cx / h)) - r, int(np.floor(cx / h)) + r + 2) % nx
        by = np.arange(int(np.floor(cy / h)) - r, int(np.floor(cy / h)) + r + 2) % ny
        bz = np.arange(int(np.floor(cz / h)) - r, int(np.floor(cz / h)) + r + 2)
        bz = bz[(bz >= 0) & (bz < nz)]
        bx, by = np.unique(bx), np.unique(by)
        gz, gy, gx = np.meshgrid(bz, by, bx, indexing="ij")
        gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
        dx = _min_image(gx * h - cx, Lx)
        dy = _min_image(gy * h - cy, Ly)
        dz = gz * h - cz
        d2 = dx * dx + dy * dy + dz * dz
        keep = d2 < cutoff * cutoff
        gidx = (gx + nx * (gy + ny * gz))[keep]
        order = np.argsort(gidx, kind="stable")
        gidx = gidx[order]
        dx, dy, dz, d2 = (a[keep][order] for a in (dx, dy, dz, d2))
        g = np.exp(-d2 / (2.0 * width * width))
        chans = np.stack([g, dx / width * g, dy / width * g, dz / width * g], axis=1)
        norms = np.sqrt((chans * chans).sum(axis=0))
        chans = chans / norms
        idx_all.append(gidx.astype(np.int64))
        p_all.append(chans)
        ptr.append(ptr[-1] + gidx.size)
        ds, dp = rng.uniform(-1.0, 1.0, size=2)
        dvals.append([ds, dp, dp, dp])
    if not centres.shape[0]:
        return (np.zeros(1, np.int64), np.zeros(0, np.int64),
                np.zeros((0, N_PROJ)), np.zeros((0, N_PROJ)))
    return (np.asarray(ptr, np.int64), np.concatenate(idx_all),
            np.ascontiguousarray(np.concatenate(p_all)), np.asarray(dvals, np.float64))


def no_projectors():
    return (np.zeros(1, np.int64), np.zeros(0, np.int64),
            np.zeros((0, N_PROJ)), np.zeros((0, N_PROJ)))


def energies(lo, hi, K, eta):
    """z_k = E_k + i*eta with E_k = linspace(lo, hi, K) (endpoints included)."""
    return np.linspace(lo, hi, K) + 1j * eta


def boundary_points(nx, ny, nz, rng, n_bottom, n_top):
    """Distinct seeded grid points on plane iz=0 (n_bottom) and iz=nz-1 (n_top)."""
    nxy = nx * ny
    out = []
    if n_bottom:
        out.append(np.sort(rng.choice(nxy, n_bottom, replace=False)))
    if n_top:
        out.append(np.sort(rng.choice(nxy, n_top, replace=False)) + nxy * (nz - 1))
    return np.concatenate(out).astype(np.int64) if out else np.zeros(0, np.int64)


def make_problem(name, nx, ny, nz, h, nf, n_atoms, projectors, K, eta, elo, ehi,
                 n_bottom, n_top, seed, tol=1e-10, centres=None, s_idx=None):
    """General builder: seeded Gaussian atoms, optional projectors, shifts, RHS set."""
    rng = np.random.default_rng(seed)
    if centres is None:
        centres = np.stack([rng.uniform(0, nx * h, n_atoms), rng.uniform(0, ny * h, n_atoms),
                            rng.uniform(0, nz * h, n_atoms)], axis=1) if n_atoms else np.zeros((0, 3))
    depths = rng.uniform(0.5, 2.0, centres.shape[0])
    vloc = gaussian_vloc(nx, ny, nz, h, centres, depths)
    proj = kb_projectors(nx, ny, nz, h, centres, rng) if projectors else no_projectors()
    rhs = boundary_points(nx, ny, nz, rng, n_bottom, n_top)
    return Problem(name=name, nx=nx, ny=ny, nz=nz, h=h, nf=nf,
                   coef=kinetic_coefficients(h, nf), vloc=vloc,
                   atom_ptr=proj[0], atom_idx=proj[1], atom_P=proj[2], atom_D=proj[3],
                   z=energies(elo, ehi, K, eta), rhs_idx=rhs, s_idx=s_idx, tol=tol,
                   centres=centres)


# ---------------------------------------------------------------------------
# The five named workloads.  Seeds: default_rng(1502 + c) for workload c.
# ---------------------------------------------------------------------------

def tiny_fp64():
    """16x16x24 grid (6144 points), h=0.4, nf=4, 6 Gaussians, no projectors;
    16 energies in [-0.5, 0.5] Ha, eta=1e-3; 8 RHS points on iz=0; tol 1e-10."""
    return make_problem("tiny_16x16x24", 16, 16, 24, 0.4, 4, 6, False, 16, 1e-3, -0.5, 0.5,
                        8, 0, 1502 + 1, tol=1e-10)


def medium_fp64():
    """48x48x96 grid (221,184 points), h=0.35, 40 atoms with Gaussian V_loc and
    4 KB projectors each; 128 energies in [-0.6, 0.6] Ha, eta=1e-3; 64 RHS
    (32 on iz=0, 32 on iz=nz-1)."""
    return make_problem("medium_48x48x96", 48, 48, 96, 0.35, 4, 40, True, 128, 1e-3, -0.6, 0.6,
                        32, 32, 1502 + 2, tol=1e-8)


def tiny_mixed():
    """Same Hamiltonian as tiny_fp64; 256 energies, all 256 points of iz=0 as RHS."""
    p = tiny_fp64()
    nxy = p.nx * p.ny
    return p.with_(name="tiny_mixed_16x16x24", z=energies(-0.5, 0.5, 256, 1e-3),
                   rhs_idx=np.arange(nxy, dtype=np.int64), tol=1e-8)


def peapod_large():
    """64x64x160 grid (655,360 points), h=0.4; 400 atoms on a 12.850 bohr cylinder
    around the box axis plus 60 on a 6.614 bohr sphere at the box centre, each
    with Gaussian V_loc and 4 KB projectors; 512 energies in [-0.5, 0.5] Ha,
    eta=5e-4; 512 RHS on iz=0 and 512 on iz=nz-1."""
    nx = ny = 64
    nz = 160
    h = 0.4
    rng = np.random.default_rng(1502 + 4)
    L, Lz = nx * h, nz * h
    th = rng.uniform(0, 2 * np.pi, 400)
    zz = rng.uniform(0, Lz, 400)
    rc = 12.850
    cyl = np.stack([L / 2 + rc * np.cos(th), L / 2 + rc * np.sin(th), zz], axis=1)
    cyl[:, 0] %= L
    cyl[:, 1] %= L
    v = rng.normal(size=(60, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    sph = np.array([L / 2, L / 2, Lz / 2]) + 6.614 * v
    centres = np.concatenate([cyl, sph])
    return make_problem("peapod_64x64x160", nx, ny, nz, h, 4, 0, True, 512, 5e-4, -0.5, 0.5,
                        512, 512, 1502 + 4, tol=1e-8, centres=centres)


def batched_regions():
    """12 regions 32x32x(48+16r), nz_r Gaussian atoms each (one per 1024 points),
    no projectors; K_r = 64+32*((5r) mod 11) energies in [-0.5, 0.5] Ha,
    eta=1e-3; R_r = 32*(1+(7r mod 8)) RHS, half on each boundary plane."""
    out = []
    for r in range(12):
        nz = 48 + 16 * r
        K = 64 + 32 * ((5 * r) % 11)
        R = 32 * (1 + (7 * r) % 8)
        out.append(make_problem(f"region{r}_32x32x{nz}", 32, 32, nz, 0.4, 4, nz, False, K, 1e-3,
                                -0.5, 0.5, R // 2, R // 2, 1502 + 5 + 100 * r, tol=1e-8))
    return out


WORKLOADS = {
    "tiny_fp64": tiny_fp64,
    "medium_fp64": medium_fp64,
    "tiny_mixed": tiny_mixed,
    "peapod_large": peapod_large,
}


# ---------------------------------------------------------------------------
# Electrodes: synthetic semi-infinite leads and their self-energies.
#
# The perturbed Green's function of the transition region needs the lead
# self-energies Sigma_L(z_0; Z) and Sigma_R(z_{m+1}; Z) (Sec. 2B, Eqs. 10-11).
# In the paper they come from the electrode calculation; here they are inputs
# built for ideal wires: the lead continues the transition region's grid and
# finite-difference operator along z with a constant potential v_lead and no
# projectors.  With half-width nf, nf consecutive x-y planes form one principal
# layer, so the boundary blocks z_0 and z_{m+1} are the first and last nf planes
# of the region (M = nf*nx*ny rows each, plane-major within the block, i.e. the
# grid order).
#
# Periodic x and y make every transverse Fourier mode q an independent
# one-dimensional chain of nf x nf layer blocks; the surface Green's function
# of each chain comes from the decimation iteration of Lopez Sancho, Lopez
# Sancho and Rubio (J. Phys. F 15, 851 (1985)), and the real-space block is the
# inverse transverse Fourier transform of the per-mode result.
# ---------------------------------------------------------------------------

def transverse_energies(nx, ny, coef):
    """eps(q) = sum_axis [c_0 + 2 sum_d c_d cos(d q)] over the nx*ny transverse modes.

    Returns eps [nx*ny] in the order q = (mx, my) -> mx + nx*my."""
    nf = coef.shape[1] - 1
    qx = 2 * np.pi * np.arange(nx) / nx
    qy = 2 * np.pi * np.arange(ny) / ny
    ex = coef[0, 0] + 2 * sum(coef[0, d] * np.cos(d * qx) for d in range(1, nf + 1))
    ey = coef[1, 0] + 2 * sum(coef[1, d] * np.cos(d * qy) for d in range(1, nf + 1))
    return (ex[None, :] + ey[:, None]).ravel()


def lead_layer_blocks(coef):
    """Layer blocks of the z chain: t00 [nf,nf] (within a layer) and t01 [nf,nf].

    t01[p, q] couples plane p of layer l to plane q of layer l+1, whose distance
    is nf + q - p; it is nonzero for q <= p."""
    nf = coef.shape[1] - 1
    cz = coef[2]
    t00 = np.zeros((nf, nf))
    t01 = np.zeros((nf, nf))
    for p in range(nf):
        for q in range(nf):
            t00[p, q] = cz[abs(p - q)]
            d = nf + q - p
            if d <= nf:
                t01[p, q] = cz[d]
    return t00, t01


def _surface_gf(zeta, t00, tc, max_iter=200):
    """Surface Green's function of a semi-infinite chain, one per row of zeta.

    The chain is layer 0, 1, 2, ... with on-site block t00 + (diagonal shift)
    and block tc coupling layer l to layer l+1 (its transpose couples back).
    zeta [nq] holds Z - shift per mode.  Decimation: every pass removes every
    other layer, squaring the effective coupling."""
    nf = t00.shape[0]
    nq = zeta.shape[0]
    eye = np.eye(nf)
    a = np.broadcast_to(tc.astype(np.complex128), (nq, nf, nf)).copy()
    b = np.broadcast_to(tc.T.astype(np.complex128), (nq, nf, nf)).copy()
    es = np.broadcast_to(t00.astype(np.complex128), (nq, nf, nf)).copy()
    e = es.copy()
    zI = zeta[:, None, None] * eye
    scale = max(1.0, float(np.abs(tc).max()))
    for _ in range(max_iter):
        g = np.linalg.inv(zI - e)
        ag = a @ g
        bg = b @ g
        agb = ag @ b
        es = es + agb
        e = e + agb + bg @ a
        a = ag @ a
        b = bg @ b
        if max(np.abs(a).max(), np.abs(b).max()) < 1e-15 * scale:
            break
    else:
        raise RuntimeError("lead decimation did not converge (Im Z too small?)")
    return np.linalg.inv(zI - es)


def lead_self_energies(nx, ny, coef, z, v_lead=0.0):
    """Sigma_L(z_0; Z_k), Sigma_R(z_{m+1}; Z_k) for ideal leads, [K, M, M] each.

    Row/column order inside a block: xy + nx*ny*p for plane p = 0..nf-1 of the
    block (grid order).  Both are complex symmetric.  Sigma_R = t01 g_R t01^T
    with g_R the surface block of the right lead (extending to +z);
    Sigma_L = t01^T g_L t01 with g_L that of the left lead (extending to -z)."""
    nf = coef.shape[1] - 1
    nxy = nx * ny
    t00, t01 = lead_layer_blocks(coef)
    eps = transverse_energies(nx, ny, coef)
    ix = np.arange(nx)
    iy = np.arange(ny)
    rx = (ix[None, :] + 0 * iy[:, None]).ravel()
    ry = (0 * ix[None, :] + iy[:, None]).ravel()
    qx = 2 * np.pi * (np.arange(nxy) % nx) / nx
    qy = 2 * np.pi * (np.arange(nxy) // nx) / ny
    # F[r, q] = exp(i q.r) / sqrt(nxy): unitary transverse Fourier basis
    F = np.exp(1j * (rx[:, None] * qx[None, :] + ry[:, None] * qy[None, :])) / np.sqrt(nxy)
    z = np.atleast_1d(np.asarray(z, np.complex128))
    M = nf * nxy
    sig_l = np.empty((z.size, M, M), np.complex128)
    sig_r = np.empty((z.size, M, M), np.complex128)
    for k, zk in enumerate(z):
        zeta = zk - eps - v_lead
        gR = _surface_gf(zeta, t00, t01)
        gL = _surface_gf(zeta, t00, t01.T)
        sR = t01 @ gR @ t01.T        # [nq, nf, nf]
        sL = t01.T @ gL @ t01
        for out, s in ((sig_r, sR), (sig_l, sL)):
            # block (p, p') = F diag_q(s[q, p, p']) F^H
            for p in range(nf):
                for pp in range(nf):
                    out[k, p * nxy:(p + 1) * nxy, pp * nxy:(pp + 1) * nxy] = \
                        (F * s[:, p, pp][None, :]) @ F.conj().T
    return sig_l, sig_r


def obm_indices(nx, ny, nz, nf, extra=None):
    """Grid indices of the left boundary block (planes 0..nf-1), the right block
    (planes nz-nf..nz-1) and optional extra rows, in that order."""
    nxy = nx * ny
    M = nf * nxy
    n = nxy * nz
    if nz < 2 * nf:
        raise ValueError("the two boundary blocks overlap: need nz >= 2*nf")
    parts = [np.arange(M), np.arange(n - M, n)]
    if extra is not None and len(extra):
        parts.append(np.asarray(extra, np.int64))
    return np.concatenate(parts).astype(np.int64)


def interior_centres(nx, ny, nz, h, nf, n_atoms, rng, margin=1.5):
    """Atom centres kept at least `margin` bohr away from the two boundary blocks
    (all at the middle plane's height when the region is too short for that)."""
    zlo = nf * h + margin
    zhi = (nz - nf - 1) * h - margin
    if zhi < zlo:
        zlo = zhi = 0.5 * (nz - 1) * h
    return np.stack([rng.uniform(0, nx * h, n_atoms), rng.uniform(0, ny * h, n_atoms),
                     rng.uniform(zlo, zhi, n_atoms)], axis=1)


def obm_wire(nx=8, ny=8, nz=32, h=0.4, n_atoms=4, K=16, eta=1e-3, elo=0.1, ehi=3.0, seed=1502 + 7,
             projectors=True, extra_plane=True, tol=1e-10):
    """Scatterer between two ideal V=0 leads for the open-boundary matching.

    8x8x32 grid (2048 points), h=0.4, nf=4; n_atoms Gaussians with projectors
    away from the boundary blocks; K energies in [0.1, 3.0] Ha (one to five
    open lead channels), eta=1e-3.  RHS set = rows = left block (256), right
    block (256) and, for the density of states, the middle plane (64).
    Returns (problem, M, L)."""
    rng = np.random.default_rng(seed)
    nf = 4
    centres = interior_centres(nx, ny, nz, h, nf, n_atoms, rng) if n_atoms else np.zeros((0, 3))
    p = make_problem(f"obm_wire_{nx}x{ny}x{nz}", nx, ny, nz, h, nf, 0, projectors, K, eta,
                     elo, ehi, 0, 0, seed, tol=tol, centres=centres)
    nxy = nx * ny
    extra = np.arange(nxy) + nxy * (nz // 2) if extra_plane else None
    idx = obm_indices(nx, ny, nz, nf, extra)
    return p.with_(rhs_idx=idx, s_idx=None), nf * nxy, (nxy if extra_plane else 0)
