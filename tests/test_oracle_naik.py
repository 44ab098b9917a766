"""Pins of the oracle's Naik-improved operator and its Kahler-Dirac multigrid
(Sec. 2.1, eq. "freehisq" and the spectra printed after it)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.staggered import (Lattice, dirac_matrix, dirac_matrix_naik, free_spectrum_naik, epsilon_dof,
                              gauge_rotate, gauge_matrix, NAIK_C1, NAIK_C3)
from oracle.kd import KDOperator
from oracle.mg import MGParams, LevelParams, Hierarchy, Solver
from synth import unit_gauge, u1_heatbath, gaussian_vectors, gauge_transform_field


def random_u1(dims, seed):
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(-np.pi, np.pi, size=(len(dims), int(np.prod(dims)), 1, 1)))


@pytest.mark.parametrize("dims,bc", [((8, 8), (1, -1)), ((12, 8), (1, 1)), ((8, 16), (-1, -1))])
def test_free_naik_spectrum(dims, bc):
    """Free Naik eigenvalues m +- i sqrt(sum_mu sin^2 p_mu (1 + sin^2 p_mu / 6)^2),
    each momentum once (full zone; antiperiodic directions shifted)."""
    lat = Lattice(dims, bc=bc)
    m = 0.07
    lam = np.linalg.eigvals(dirac_matrix_naik(lat, unit_gauge(dims), m).toarray())
    assert np.allclose(lam.real, m, atol=1e-12)
    assert np.allclose(np.sort(lam.imag ** 2), free_spectrum_naik(lat, m), atol=1e-11)


def test_naik_symbol_from_coefficients():
    """Per direction the free symbol is c1 sin p + c3 sin 3p = sin p (1 + sin^2 p / 6)
    for (c1, c3) = (9/8, -1/24): the printed 9/16 and 1/48 are these halved, and
    only this normalisation reproduces the printed spectrum."""
    p = np.linspace(-np.pi, np.pi, 101)
    assert np.allclose(NAIK_C1 * np.sin(p) + NAIK_C3 * np.sin(3 * p), np.sin(p) * (1 + np.sin(p) ** 2 / 6),
                       atol=1e-15)
    assert np.isclose(NAIK_C1 / 2, 9 / 16) and np.isclose(-NAIK_C3 / 2, 1 / 48)


def test_naik_reduces_to_staggered():
    """c1 = 1, c3 = 0 is eq. "staggeredD"."""
    dims = (8, 12)
    lat = Lattice(dims)
    U = random_u1(dims, 3)
    D0 = dirac_matrix(lat, U, 0.3)
    D1 = dirac_matrix_naik(lat, U, 0.3, c1=1.0, c3=0.0)
    assert abs(D0 - D1).max() < 1e-15


@pytest.mark.parametrize("nc", [1, 3])
def test_naik_symmetries_and_gauge_covariance(nc):
    """D - m anti-Hermitian, eps D eps = D^dag (three-link hops join opposite
    parities), and D[U^g] = G D[U] G^dag with the long links built from U^g."""
    dims = (8, 8) if nc == 1 else (4, 4, 4, 8)
    lat = Lattice(dims, ncolor=nc)
    if nc == 1:
        U = random_u1(dims, 5)
    else:
        U = gauge_transform_field(lat.volume * lat.nd, 3, 6).reshape(lat.nd, lat.volume, 3, 3)
    m = 0.2
    D = dirac_matrix_naik(lat, U, m)
    H = (D - m * sp.identity(lat.ndof)).toarray()
    assert np.abs(H + H.conj().T).max() < 1e-14
    E = sp.diags(epsilon_dof(lat))
    assert abs(E @ D @ E - D.conj().T).max() < 1e-14
    g = gauge_transform_field(lat.volume, nc, 7)
    G = gauge_matrix(lat, g)
    Dg = dirac_matrix_naik(lat, gauge_rotate(lat, U, g), m)
    assert abs(Dg - G @ D @ G.conj().T).max() < 1e-13


def test_naik_kd_block_and_c():
    """Sec. 2.1: the Naik KD block is the plain one with its hops rescaled
    (B_Naik - m = (9/8)(B - m)); the new terms sit in C only, which is no
    longer a multiple of a unitary (C^dag C not proportional to 1), and half
    of the three-link hops join blocks of the same parity."""
    dims = (8, 8)
    lat = Lattice(dims)
    U = random_u1(dims, 8)
    m = 0.15
    kd = KDOperator(lat, U, m)
    kn = KDOperator(lat, U, m, naik=True)
    I = sp.identity(lat.volume)
    assert abs((kn.B - m * I) - NAIK_C1 * (kd.B - m * I)).max() < 1e-15
    CC = (kn.C.conj().T @ kn.C).toarray()
    assert np.abs(CC - np.mean(np.diag(CC)) * np.eye(lat.volume)).max() > 1e-3
    assert not kn.has_schur and abs(kn.A[kn.even][:, kn.even] - sp.identity(kn.even.size)).max() > 1e-3


def test_free_massless_kd_naik_spectrum():
    """The massless free KD-Naik spectrum printed for d = 2:
    lambda = 1 - a +- i sqrt(1 - a^2 - 2x [S2 - S1 + x (S3 - 1)]),
    a = (1 - x) S1 + x S2, S_n = (1/2) sum_mu cos(n P_mu), x = (-1/48)/(9/16),
    over the KD-block momenta P, each value twice."""
    L = 8
    lat = Lattice((L, L), bc=(1, 1))
    kd = KDOperator(lat, unit_gauge((L, L)), 0.0, naik=True)
    lam = np.linalg.eigvals(kd.A.toarray())
    x = (-1 / 48) / (9 / 16)
    P = 2 * np.pi * np.arange(L // 2) / (L // 2)
    ref = []
    for P0 in P:
        for P1 in P:
            S = lambda n: 0.5 * (np.cos(n * P0) + np.cos(n * P1))
            a = (1 - x) * S(1) + x * S(2)
            im = 1j * np.sqrt(complex(1 - a * a - 2 * x * (S(2) - S(1) + x * (S(3) - 1))))
            ref += [1 - a + im, 1 - a + im, 1 - a - im, 1 - a - im]
    ref = np.array(ref)
    assert np.allclose(np.sort(lam.real), np.sort(ref.real), atol=1e-10)
    assert np.allclose(np.sort(lam.imag ** 2), np.sort(ref.imag ** 2), atol=1e-10)
    # the plain operator's circle is lost: |lambda - 1| is not constant
    assert np.ptp(np.abs(lam - 1)) > 1e-2


@pytest.mark.parametrize("levels", [[((4, 4), 8)], [((2, 2), 8), ((2, 2), 8)]])
def test_naik_kd_multigrid_solve(levels):
    """KD-MG on the Naik operator (fine FGCR on the full A, x = B^-1 y; the
    K-cycle and coarse levels as for the plain operator): true residual
    <= 1e-10 and the dense-LU solution to 1e-8; the coarse operator is still
    a nearest-neighbour stencil (three-link hops reach at most the
    neighbouring aggregate)."""
    dims = (32, 32)
    U, _ = u1_heatbath(dims, 6.0, 60, 17)
    lat = Lattice(dims)
    m = 0.05
    psi0 = []
    n, ncs = lat.ndof, None
    for k, (agg, nv) in enumerate(levels):
        psi0.append(gaussian_vectors(nv, n, 17, tag=1 + k))
        ncs = lat.volume // int(np.prod([2 * a for a in agg])) if k == 0 else ncs // int(np.prod(agg))
        n = ncs * 2 * nv
    h = Hierarchy(lat, U, m, MGParams(levels=[LevelParams(a, nv) for a, nv in levels]), psi0, naik=True)
    assert not h.fine_schur
    b = gaussian_vectors(1, lat.ndof, 18)[0]
    x, info = Solver(h).solve(b, 1e-10)
    D = dirac_matrix_naik(lat, U, m)
    assert info["converged"] and np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-10
    xd = np.linalg.solve(D.toarray(), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    assert info["outer_its"] < 60, info
    # nearest-neighbour coarse stencil: coarse sites farther than one apart do not couple
    A1 = h.ops[1].tocoo()
    cd = h.aggr[0].coarse_dims
    nd1 = 2 * levels[0][1]
    z0, z1 = (A1.row // nd1) % cd[0], (A1.row // nd1) // cd[0]
    w0, w1 = (A1.col // nd1) % cd[0], (A1.col // nd1) // cd[0]
    d0 = np.minimum((z0 - w0) % cd[0], (w0 - z0) % cd[0])
    d1 = np.minimum((z1 - w1) % cd[1], (w1 - z1) % cd[1])
    assert np.all(d0 + d1 <= 1)
