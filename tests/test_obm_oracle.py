"""Pins of the open-boundary oracle (perturbed blocks, transmission, DOS) and of the
synthetic lead self-energies, against things other than themselves (CPU only).

What fixes each expected value:
  * the closed-form surface Green's function of a nearest-neighbour chain and the
    closed-form transmission of a single-site impurity on it,
  * channel counting from the lead dispersion: an ideal wire transmits exactly
    one unit per propagating transverse mode,
  * the Green's function of the infinite ideal wire, summed over a long periodic
    ring in the Fourier basis (no leads, no self-energies),
  * the corner block of a long finite chain inverted densely (brute force for
    the surface Green's function of a semi-infinite lead),
  * exact identities of a resolvent with self-energies: complex symmetry,
    reciprocity of T, and i(G - G^dagger) = G (Gamma_L + Gamma_R + 2 eta) G^dagger.
"""
import numpy as np
import pytest

from oracle import obm as O
from paper_1502_00081_amd import workload as W
from tests import dense_ref as D


def chain_problem(nz, h, v=None, nf=1, nx=1, ny=1, n_atoms=0, projectors=False, seed=3):
    p = W.make_problem("chain", nx, ny, nz, h, nf, n_atoms, projectors, 1, 1e-3, 0.0, 1.0, 0, 0,
                       seed)
    if v is not None:
        p = p.with_(vloc=np.asarray(v, np.float64))
    return p


def blocks(p):
    M = p.nf * p.nx * p.ny
    return M, np.arange(M), np.arange(p.n - M, p.n)


def solve_all(p, z, v_lead=0.0, H=None):
    """Perturbed G_T on (left block, right block) and T for each energy."""
    sl, sr = W.lead_self_energies(p.nx, p.ny, p.coef, z, v_lead)
    M, left, right = blocks(p)
    idx = np.concatenate([left, right])
    G = O.perturbed_green(p, z, sl, sr, idx, H=H)
    T = np.array([O.transmission(sl[k], sr[k], G[k][M:, :M]) for k in range(len(z))])
    return G, T, sl, sr


def test_surface_gf_matches_nearest_neighbour_closed_form():
    """nf = 1, one transverse mode: g = (zeta - sqrt(zeta^2 - 4 t^2)) / (2 t^2), the root
    with Im g < 0; Sigma = t^2 g on both sides."""
    h = 0.7
    coef = W.kinetic_coefficients(h, 1)
    t = coef[2, 1]
    eps0 = coef[2, 0] + (coef[0, 0] + 2 * coef[0, 1]) + (coef[1, 0] + 2 * coef[1, 1])
    z = np.array([0.3 + 1e-3j, 1.1 + 1e-6j, -0.4 + 0.05j, 5.0 + 1e-4j])
    sl, sr = W.lead_self_energies(1, 1, coef, z)
    for k, zk in enumerate(z):
        zeta = zk - eps0
        roots = [(zeta + s * np.sqrt(zeta * zeta - 4 * t * t)) / (2 * t * t) for s in (1, -1)]
        g = [r for r in roots if r.imag < 0][0]
        assert abs(sl[k, 0, 0] - t * t * g) < 1e-12 * abs(t * t * g) + 1e-14
        assert abs(sr[k, 0, 0] - t * t * g) < 1e-12 * abs(t * t * g) + 1e-14


@pytest.mark.parametrize("nf,nx,ny,h", [(2, 2, 2, 0.6), (4, 2, 3, 0.7)])
def test_self_energy_matches_long_chain_brute_force(nf, nx, ny, h):
    """Surface blocks of a long Dirichlet chain of layers (dense inverse) converge to the
    semi-infinite leads' at Im Z = 0.3; Sigma_R = B g_R B^T, Sigma_L = B^T g_L B with B
    the coupling block between neighbouring layers."""
    coef = W.kinetic_coefficients(h, nf)
    nxy = nx * ny
    M = nf * nxy
    n_layers = 120
    nzc = n_layers * nf
    Hc = (np.kron(np.eye(nzc), np.kron(np.eye(ny), D.circulant_1d(nx, coef[0])))
          + np.kron(np.eye(nzc), np.kron(D.circulant_1d(ny, coef[1]), np.eye(nx)))
          + np.kron(D.toeplitz_dirichlet_1d(nzc, coef[2]), np.eye(nxy)))
    # B couples the last M rows of the region to the first M rows of the next layer:
    # it is the (0, 1) layer block of the same Kronecker sum
    B = Hc[:M, M:2 * M]
    z = np.array([0.4 + 0.3j, 2.0 + 0.3j])
    sl, sr = W.lead_self_energies(nx, ny, coef, z)
    for k, zk in enumerate(z):
        G = np.linalg.inv(zk * np.eye(Hc.shape[0]) - Hc)
        gR = G[:M, :M]          # first layer of a chain extending to +z
        gL = G[-M:, -M:]        # last layer of a chain extending to -z
        ref_r = B @ gR @ B.T
        ref_l = B.T @ gL @ B
        assert np.abs(sr[k] - ref_r).max() < 1e-10 * np.abs(ref_r).max()
        assert np.abs(sl[k] - ref_l).max() < 1e-10 * np.abs(ref_l).max()


@pytest.mark.parametrize("U", [0.3, -1.2, 2.5])
def test_single_impurity_transmission_closed_form(U):
    """Chain with hopping t, one site of potential U: T = (2t sin k)^2 / ((2t sin k)^2 + U^2)
    at E = eps0 + 2t cos k (t < 0 here)."""
    h = 1.0
    nz = 7
    v = np.zeros(nz)
    v[3] = U
    p = chain_problem(nz, h, v)
    t = p.coef[2, 1]
    eps0 = p.coef[2, 0]
    ks = np.array([0.3, 0.9, 1.6, 2.4])
    E = eps0 + 2 * t * np.cos(ks)
    z = E + 1e-10j
    _, T, _, _ = solve_all(p, z)
    ref = (2 * t * np.sin(ks)) ** 2 / ((2 * t * np.sin(ks)) ** 2 + U * U)
    assert np.abs(T.imag).max() < 1e-9
    assert np.allclose(T.real, ref, rtol=0, atol=1e-7), (T.real, ref)


def open_channels(coef, nx, ny, E):
    """Propagating modes at energy E: crossings of E with eps_q + Ez(k), k in (0, pi)."""
    eps = W.transverse_energies(nx, ny, coef)
    k = np.linspace(0, np.pi, 40001)
    ez = D.fd_symbol(coef[2], k)
    n = 0
    for e in eps:
        s = np.sign(ez + e - E)
        n += int(np.count_nonzero(s[1:] != s[:-1]))
    return n


def test_ideal_wire_transmits_one_per_open_channel():
    """V = 0 everywhere: the transition region is a piece of the leads, so T(E) is the
    number of propagating transverse modes (here 1..5 over the energy range)."""
    h = 0.5
    p = chain_problem(8, h, nf=4, nx=4, ny=4)
    p = p.with_(vloc=np.zeros(p.n))
    eps = W.transverse_energies(p.nx, p.ny, p.coef)
    top = D.fd_symbol(p.coef[2], np.pi)
    edges = np.concatenate([eps, eps + top])
    E = np.array([0.2, 1.0, 2.6, 3.4, 6.0, 9.0])
    assert np.min(np.abs(E[:, None] - edges[None, :])) > 0.05
    _, T, _, _ = solve_all(p, E + 1e-9j)
    n_ch = np.array([open_channels(p.coef, p.nx, p.ny, e) for e in E])
    assert n_ch.min() >= 1 and n_ch.max() >= 3
    assert np.abs(T.imag).max() < 1e-8
    assert np.allclose(T.real, n_ch, atol=2e-6), (T.real, n_ch)


def test_ideal_wire_green_function_equals_infinite_wire():
    """V = 0: G_T restricted to the region is the infinite wire's Green's function, summed
    per transverse mode over a long periodic ring, G_q(d) = (1/n) sum_k e^{ikd}/(Z - eps_q -
    Ez(k))."""
    h = 0.5
    nx, ny, nf, nz = 2, 3, 4, 9
    p = chain_problem(nz, h, nf=nf, nx=nx, ny=ny)
    p = p.with_(vloc=np.zeros(p.n))
    z = np.array([0.8 + 0.05j, 3.0 + 0.05j])
    G, _, _, _ = solve_all(p, z)
    nxy = nx * ny
    M = nf * nxy
    eps = W.transverse_energies(nx, ny, p.coef)
    q_x = 2 * np.pi * (np.arange(nxy) % nx) / nx
    q_y = 2 * np.pi * (np.arange(nxy) // nx) / ny
    n_ring = 20000
    kk = 2 * np.pi * np.arange(n_ring) / n_ring
    ez = D.fd_symbol(p.coef[2], kk)
    # rows/cols of the two blocks: grid index -> (x, y, plane)
    idx = np.concatenate([np.arange(M), np.arange(p.n - M, p.n)])
    rx, ry, rz = idx % nx, (idx // nx) % ny, idx // nxy
    for k, zk in enumerate(z):
        dz = np.arange(-(nz - 1), nz)
        gq = np.empty((nxy, dz.size), np.complex128)
        for q in range(nxy):
            w = 1.0 / (zk - eps[q] - ez)
            gq[q] = (np.exp(1j * np.outer(dz, kk)) @ w) / n_ring
        ref = np.zeros((idx.size, idx.size), np.complex128)
        for q in range(nxy):
            ph = np.exp(1j * (q_x[q] * rx + q_y[q] * ry))
            ref += np.outer(ph, ph.conj()) * gq[q][(rz[:, None] - rz[None, :]) + nz - 1]
        ref /= nxy
        assert np.abs(G[k] - ref).max() < 1e-9 * np.abs(ref).max()


def scatterer():
    rng = np.random.default_rng(11)
    nx = ny = 4
    nz, h, nf = 12, 0.45, 4
    centres = W.interior_centres(nx, ny, nz, h, nf, 2, rng, margin=0.5)
    p = W.make_problem("scatterer", nx, ny, nz, h, nf, 0, True, 1, 1e-3, 0.0, 1.0, 0, 0, 5,
                       centres=centres)
    return p


def test_scatterer_identities():
    """Complex symmetry of G_T, real T, reciprocity T(L->R) = T(R->L), 0 <= T <= channels,
    and i (G - G^dagger) = G (Gamma_L + Gamma_R) G^dagger on the boundary rows (eta -> 0)."""
    p = scatterer()
    H = O.dense_h(p)
    E = np.array([0.3, 1.5, 2.9])
    z = E + 1e-9j
    sl, sr = W.lead_self_energies(p.nx, p.ny, p.coef, z)
    M, left, right = blocks(p)
    idx = np.concatenate([left, right])
    G = O.perturbed_green(p, z, sl, sr, idx, H=H)
    for k in range(E.size):
        g = G[k]
        assert np.abs(g - g.T).max() < 1e-10 * np.abs(g).max()
        T = O.transmission(sl[k], sr[k], g[M:, :M])
        T_back = O.transmission(sr[k], sl[k], g[:M, M:])
        assert abs(T.imag) < 1e-8
        assert abs(T - T_back) < 1e-8
        assert -1e-9 < T.real <= open_channels(p.coef, p.nx, p.ny, E[k]) + 1e-9
        gam = np.zeros((2 * M, 2 * M), np.complex128)
        gam[:M, :M] = O.gamma(sl[k])
        gam[M:, M:] = O.gamma(sr[k])
        lhs = 1j * (g - g.conj().T)
        rhs = g @ gam @ g.conj().T
        assert np.abs(lhs - rhs).max() < 1e-7 * np.abs(lhs).max()


def test_dense_h_matches_kronecker_assembly():
    """The oracle's dense H_T (stencil columns) equals an independent Kronecker-sum build."""
    p = scatterer()
    assert np.abs(O.dense_h(p) - D.dense_h(p)).max() < 1e-12


def test_dos_is_nonnegative_and_obeys_the_sum_rule():
    """-Im G_ii / pi >= 0, and each site's spectral weight integrates to one over all
    energies (the 1/Z decay of a resolvent; leads only redistribute it): over [-10, 12] Ha
    with eta = 0.02 the Lorentzian tails outside the window hold well under 1 %."""
    p = chain_problem(6, 1.0, nf=1)
    p = p.with_(vloc=np.linspace(-0.2, 0.3, 6))
    E = np.linspace(-10.0, 12.0, 8001)
    z = E + 0.02j
    sl, sr = W.lead_self_energies(p.nx, p.ny, p.coef, z)
    H = O.dense_h(p)
    G = O.perturbed_green(p, z, sl, sr, np.arange(p.n), H=H)
    rho = np.array([O.dos(G[k]) for k in range(E.size)])
    assert rho.min() > 0
    total = np.trapezoid(rho, E)
    assert abs(total - p.n) < 0.005 * p.n, total
