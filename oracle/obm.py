"""CPU FP64 oracle for the open-boundary step: perturbed Green's function blocks,
Fisher-Lee transmission and the local density of states.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's CPU
baseline leg may use it.  It never imports the GPU library.

The perturbed Green's function of the transition region is, by definition, the
inverse of the finite matrix of Sec. 2B, Eq. 13: Z - H_T with the left lead's
self-energy added to the block of the first principal layer z_0 and the right
lead's to the block of the last layer z_{m+1}.  This module builds that matrix
densely (H_T column by column from the pinned stencil oracle) and inverts it
with a library solve; there is no blocking, no use of the unperturbed Green's
function and no matching algebra, so it is independent of the shortcut of
Sec. 3B (Eqs. 18-24) that the GPU path takes.

Functions:
  dense_h(op)                                 H_T as a dense [N, N] array (Sec. 2A, Eq. 4)
  perturbed_green(op, z, sig_l, sig_r, idx)   G_T(Z)[idx, idx] from Eq. 13
  transmission(sig_l, sig_r, g_r0)            T(E), Eq. 14 with Gamma of Eq. 16
  dos(g_block)                                -Im tr G / pi
Block conventions: sig_l and sig_r are [M, M] on the first and last M grid
indices (the nf planes nearest each lead, grid order); g_r0 is the block
G_T(z_{m+1}, z_0) (rows: right block, columns: left block).
"""
from __future__ import annotations

import numpy as np

from . import apply_h


def dense_h(op):
    """H_T assembled by applying the stencil oracle to every unit vector."""
    n = op.nx * op.ny * op.nz
    H = np.empty((n, n))
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[j] = 1.0
        H[:, j] = apply_h(op, e).real
        e[j] = 0.0
    return H


def eq13_matrix(H, z, sig_l, sig_r):
    """Z - H_T - Sigma_L (on the first M rows/columns) - Sigma_R (on the last M)."""
    n = H.shape[0]
    M = sig_l.shape[0]
    A = z * np.eye(n) - H
    A = A.astype(np.complex128)
    A[:M, :M] -= sig_l
    A[n - M:, n - M:] -= sig_r
    return A


def perturbed_green(op, z, sig_l, sig_r, idx, H=None):
    """G_T(Z_k)[idx, idx] for every energy: [K, D, D] with D = len(idx)."""
    if H is None:
        H = dense_h(op)
    n = H.shape[0]
    z = np.atleast_1d(z)
    idx = np.asarray(idx)
    out = np.empty((z.size, idx.size, idx.size), np.complex128)
    for k, zk in enumerate(z):
        A = eq13_matrix(H, zk, sig_l[k], sig_r[k])
        E = np.zeros((n, idx.size), np.complex128)
        E[idx, np.arange(idx.size)] = 1.0
        G = np.linalg.solve(A, E)          # columns idx of G_T
        out[k] = G[idx, :]
    return out


def gamma(sig):
    """Coupling matrix i (Sigma - Sigma^dagger) (Eq. 16)."""
    return 1j * (sig - sig.conj().T)


def transmission(sig_l, sig_r, g_r0):
    """Fisher-Lee T = Tr[Gamma_L G^a(z_0, z_{m+1}) Gamma_R G^r(z_{m+1}, z_0)] (Eq. 14).

    G^a(z_0, z_{m+1}) is the conjugate transpose of G^r(z_{m+1}, z_0).  Returns
    the complex trace (its imaginary part vanishes up to rounding)."""
    return np.trace(gamma(sig_l) @ g_r0.conj().T @ gamma(sig_r) @ g_r0)


def dos(g_block):
    """-Im tr G / pi over the rows of a diagonal block."""
    return -np.trace(g_block).imag / np.pi
