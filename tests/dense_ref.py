"""Independent dense constructions used to pin the oracle (test helpers).

The operator is assembled here as a Kronecker sum of one-dimensional matrices
(circulant along the periodic x and y axes, banded Toeplitz truncated to the
transition region along z) plus diag(V) plus dense P D P^T blocks -- a
different construction from the oracle's point-by-point stencil loop.  The
closed forms below come from diagonalising those one-dimensional matrices
analytically (Fourier modes along periodic axes, sine modes for the
nearest-neighbour Dirichlet chain).
"""
import numpy as np


def circulant_1d(n, c):
    """n x n periodic matrix with entries c[|k|] on offsets k = -nf..nf (wrapping, summed)."""
    nf = len(c) - 1
    T = np.zeros((n, n))
    for i in range(n):
        for k in range(-nf, nf + 1):
            T[i, (i + k) % n] += c[abs(k)]
    return T


def toeplitz_dirichlet_1d(n, c):
    """n x n banded Toeplitz matrix with entries c[|k|], truncated at both ends."""
    nf = len(c) - 1
    T = np.zeros((n, n))
    for i in range(n):
        for k in range(-nf, nf + 1):
            if 0 <= i + k < n:
                T[i, i + k] += c[abs(k)]
    return T


def dense_h(p):
    """Dense H for index order i = ix + nx*(iy + ny*iz) (z slowest)."""
    Ix, Iy, Iz = np.eye(p.nx), np.eye(p.ny), np.eye(p.nz)
    Tx = circulant_1d(p.nx, p.coef[0])
    Ty = circulant_1d(p.ny, p.coef[1])
    Tz = toeplitz_dirichlet_1d(p.nz, p.coef[2])
    H = (np.kron(Iz, np.kron(Iy, Tx)) + np.kron(Iz, np.kron(Ty, Ix))
         + np.kron(Tz, np.kron(Iy, Ix)))
    H += np.diag(p.vloc)
    n = p.nx * p.ny * p.nz
    for a in range(p.atom_ptr.size - 1):
        lo, hi = p.atom_ptr[a], p.atom_ptr[a + 1]
        U = np.zeros((n, p.atom_P.shape[1]))
        U[p.atom_idx[lo:hi], :] = p.atom_P[lo:hi]
        H += U @ np.diag(p.atom_D[a]) @ U.T
    return H


def fd_symbol(c, kh):
    """Eigenvalue of the periodic 1-D stencil on the Fourier mode exp(i k x)."""
    return c[0] + 2.0 * sum(c[m] * np.cos(m * kh) for m in range(1, len(c)))


def greens_v0_periodic_xy(p, z, src, rows):
    """G(z)[rows, src] for V = 0, no projectors: Fourier modes in x, y and a
    dense solve of the nz x nz truncated Toeplitz block per (kx, ky)."""
    nx, ny, nz = p.nx, p.ny, p.nz
    sx, sy, sz = src % nx, (src // nx) % ny, src // (nx * ny)
    rx, ry, rz = rows % nx, (rows // nx) % ny, rows // (nx * ny)
    Tz = toeplitz_dirichlet_1d(nz, p.coef[2])
    out = np.zeros(rows.size, np.complex128)
    for mx in range(nx):
        kx = 2 * np.pi * mx / nx
        ex = fd_symbol(p.coef[0], kx)
        for my in range(ny):
            ky = 2 * np.pi * my / ny
            ey = fd_symbol(p.coef[1], ky)
            g = np.linalg.solve((z - ex - ey) * np.eye(nz) - Tz, np.eye(nz)[:, sz])
            out += np.exp(1j * (kx * (rx - sx) + ky * (ry - sy))) * g[rz]
    return out / (nx * ny)


def greens_chain_dirichlet(n, h, z, j, k):
    """Nearest-neighbour chain -1/2 (psi_{i-1} - 2 psi_i + psi_{i+1}) / h^2 on
    sites 1..n with psi_0 = psi_{n+1} = 0: sine modes, eps_m = (1 - cos(m pi/(n+1))) / h^2."""
    m = np.arange(1, n + 1)
    th = m * np.pi / (n + 1)
    eps = (1.0 - np.cos(th)) / (h * h)
    return np.sum(2.0 / (n + 1) * np.sin(th * j) * np.sin(th * k) / (z - eps))
