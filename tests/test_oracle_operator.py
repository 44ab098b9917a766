"""Pins of the oracle's operators against the paper's closed forms and exact
invariants (Sec. 2 and 2.1).  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.staggered import (Lattice, dirac_matrix, epsilon_dof, free_spectrum,
                              gauge_rotate, gauge_matrix, eta)
from oracle.kd import KDOperator, block_of_site, split_B_C
from oracle.exact import dense_solve, cg_eo, free_fft_solve
from synth import (u1_heatbath, unit_gauge, gaussian_vectors,
                   gauge_transform_field, su3_smooth_random)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_u1(dims, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=(len(dims), int(np.prod(dims)), 1, 1))
    return np.exp(1j * th)


def random_su3(dims, seed):
    V = int(np.prod(dims))
    g = gauge_transform_field(V * len(dims), 3, seed)
    return g.reshape(len(dims), V, 3, 3)


@pytest.mark.parametrize("dims,anti", [((8, 8), True), ((4, 8), True),
                                       ((6, 4), True), ((4, 4, 4), True)])
def test_free_spectrum_closed_form(dims, anti):
    """Sec. 2: free eigenvalues m +- i sqrt(sum sin^2 p_mu)."""
    lat = Lattice(dims, antiperiodic_time=anti)
    m = 0.1
    D = dirac_matrix(lat, unit_gauge(dims), m).toarray()
    lam = np.linalg.eigvals(D)
    assert np.allclose(lam.real, m, atol=1e-12)
    assert np.allclose(np.sort(lam.imag ** 2), free_spectrum(lat, m), atol=1e-11)
    # eigenvalues come in complex-conjugate pairs
    assert np.allclose(np.sort(lam.imag), np.sort(-lam.imag), atol=1e-11)


def test_free_spectrum_periodic_zero_modes():
    """Fully periodic free operator: 2^d exact modes at lambda = m."""
    lat = Lattice((8, 8), antiperiodic_time=False)
    D = dirac_matrix(lat, unit_gauge((8, 8)), 0.05).toarray()
    lam = np.linalg.eigvals(D)
    assert np.sum(np.abs(lam - 0.05) < 1e-10) == 4


@pytest.mark.parametrize("nc", [1, 3])
def test_symmetries(nc):
    """(D - m) anti-Hermitian, normal, eps-Hermitian, eps D + D eps = 2 m eps."""
    dims = (4, 6) if nc == 1 else (4, 4, 2, 4)
    lat = Lattice(dims, ncolor=nc)
    U = random_u1(dims, 1) if nc == 1 else random_su3(dims, 1)
    m = 0.3
    D = dirac_matrix(lat, U, m).toarray()
    K = D - m * np.eye(D.shape[0])
    assert np.allclose(K.conj().T, -K, atol=1e-14)
    assert np.allclose(D @ D.conj().T, D.conj().T @ D, atol=1e-13)
    E = np.diag(epsilon_dof(lat))
    assert np.allclose(E @ D @ E, D.conj().T, atol=1e-14)
    assert np.allclose(E @ D + D @ E, 2 * m * E, atol=1e-14)


@pytest.mark.parametrize("nc", [1, 3])
def test_gauge_covariance(nc):
    dims = (6, 4) if nc == 1 else (2, 2, 4, 4)
    lat = Lattice(dims, ncolor=nc)
    U = random_u1(dims, 2) if nc == 1 else random_su3(dims, 2)
    g = gauge_transform_field(lat.volume, nc, 7)
    D = dirac_matrix(lat, U, 0.2)
    Dg = dirac_matrix(lat, gauge_rotate(lat, U, g), 0.2)
    G = gauge_matrix(lat, g)
    assert abs(Dg - G @ D @ G.conj().T).max() < 1e-14


def test_free_normal_operator_is_spacing_two_laplacian():
    """Sec. 2: free D^dag D = m^2 + 1/4 sum_mu (2 - T_{2mu} - T_{-2mu})."""
    dims = (8, 6)
    lat = Lattice(dims)
    m = 0.2
    D = dirac_matrix(lat, unit_gauge(dims), m)
    n = lat.volume
    L = sp.identity(n) * (m * m)
    for mu in range(2):
        f1, s1 = lat.neighbour(mu, +1)
        f2 = f1[f1]
        s2 = s1 * s1[f1]
        T2 = sp.coo_matrix((s2, (np.arange(n), f2)), shape=(n, n))
        L = L + 0.25 * (2 * sp.identity(n) - T2 - T2.T)
    assert abs(D.conj().T @ D - L).max() < 1e-14


@pytest.mark.parametrize("dims", [(8, 8), (16, 12), (4, 4, 4, 8)])
def test_free_fft_solve(dims):
    lat = Lattice(dims)
    b = gaussian_vectors(1, lat.ndof, 3)[0]
    m = 0.05
    x = free_fft_solve(lat, m, b)
    D = dirac_matrix(lat, unit_gauge(dims), m)
    assert np.linalg.norm(D @ x - b) / np.linalg.norm(b) < 1e-12
    if lat.volume <= 256:
        assert np.allclose(x, dense_solve(lat, unit_gauge(dims), m, b), atol=1e-10)


def test_printed_kd_block():
    """Sec. 2.1 eq. localblock, read with the +1/2 hopping of eq. staggeredD:
    the oracle's B equals the printed block with its off-diagonal 2x2 blocks
    negated."""
    with open(os.path.join(GOLDEN, "kd_block_2d.json")) as f:
        gold = json.load(f)
    dims = (6, 8)
    lat = Lattice(dims)
    U = random_u1(dims, 5)
    m = 0.37
    D = dirac_matrix(lat, U, m)
    B, _ = split_B_C(lat, D)
    B = B.toarray()
    for n0, n1 in [(0, 0), (1, 2), (2, 3)]:
        c0 = (2 * n0, 2 * n1)
        pos = {"2n": c0, "2n+x": (c0[0] + 1, c0[1]), "2n+y": (c0[0], c0[1] + 1),
               "2n+x+y": (c0[0] + 1, c0[1] + 1)}
        sites = [int(lat.index(pos[s])) for s in gold["site_order"]]
        printed = np.eye(4, dtype=complex) * m
        for e in gold["entries"]:
            u = U[e["mu"], int(lat.index(pos[e["at"]])), 0, 0]
            printed[e["row"], e["col"]] = e["coeff"] * (np.conj(u) if e["dagger"] else u)
        ours = B[np.ix_(sites, sites)]
        flip = np.diag([1, 1, -1, -1])
        # negate the two off-diagonal (even-odd) 2x2 blocks
        expect = printed.copy()
        expect[:2, 2:] *= -1
        expect[2:, :2] *= -1
        assert np.allclose(ours, expect, atol=1e-15)
        # the two readings are epsilon-similar: D(-1/2) = eps D(+1/2) eps
        assert np.allclose(flip @ ours @ flip, printed, atol=1e-15)


def test_block_structure():
    dims = (8, 8)
    lat = Lattice(dims)
    U = random_u1(dims, 4)
    kd = KDOperator(lat, U, 0.1)
    # B - m is anti-Hermitian, B is block diagonal, C holds half the links
    Bd = kd.B.toarray()
    K = Bd - 0.1 * np.eye(lat.volume)
    assert np.allclose(K.conj().T, -K, atol=1e-15)
    blk = block_of_site(lat)
    r, c = kd.B.nonzero()
    assert np.all(blk[r] == blk[c])
    assert kd.C.nnz == (kd.D.nnz - lat.volume) // 2
    # B^-1 really inverts B
    assert abs(kd.B @ kd.Binv - sp.identity(lat.volume)).max() < 1e-13


@pytest.mark.parametrize("d,dims", [(2, (8, 8)), (4, (4, 4, 4, 4))])
def test_free_B_C_hat_unitary(d, dims):
    """Sec. 2.1 with the 1/2 hopping of eq. staggeredD: B_hat = B eps/sqrt(m^2+d/4)
    and C_hat = C eps/sqrt(d/4) square to 1."""
    lat = Lattice(dims, antiperiodic_time=False)
    m = 0.3
    kd = KDOperator(lat, unit_gauge(dims), m)
    E = sp.diags(epsilon_dof(lat))
    I = sp.identity(lat.volume)
    Bh = kd.B @ E / np.sqrt(m * m + d / 4)
    Ch = kd.C @ E / np.sqrt(d / 4)
    assert abs(Bh @ Bh - I).max() < 1e-13
    assert abs(Ch @ Ch - I).max() < 1e-13
    assert abs(Bh @ Bh.conj().T - I).max() < 1e-13


@pytest.mark.parametrize("m", [0.0, 0.25])
def test_free_kd_spectrum_circle(m):
    """Sec. 2.1: free A = 1 + rho U has eigenvalues on |lambda - 1| = rho with
    rho = sqrt(d/(d + 4 m^2)) (1/2 hopping), real parts 1 - (rho^2/d) sum cos P_mu
    over block momenta P = 2p."""
    dims = (8, 8)
    d = 2
    lat = Lattice(dims, antiperiodic_time=False)
    kd = KDOperator(lat, unit_gauge(dims), m)   # free B is invertible at m = 0
    lam = np.linalg.eigvals(kd.A.toarray())
    rho = np.sqrt(d / (d + 4 * m * m))
    assert np.allclose(np.abs(lam - 1), rho, atol=1e-12)
    ps = [2 * np.pi * np.arange(L) / L for L in dims]
    g = np.meshgrid(*ps, indexing="ij")
    re = 1 - (rho * rho / d) * sum(np.cos(2 * x) for x in g).ravel()
    assert np.allclose(np.sort(lam.real), np.sort(re), atol=1e-11)
    if m == 0:
        # massless formula lambda = 1 - c +- i sqrt(1 - c^2), c = (1/d) sum cos P
        c = (1 / d) * sum(np.cos(2 * x) for x in g).ravel()
        assert np.allclose(np.sort(lam.imag ** 2), np.sort(1 - c * c), atol=1e-10)


def test_kd_adjoint_identities():
    """Sec. 2.1 eqs. gamma5L / gamma5R and eps A^dag eps = B^-1 D."""
    dims = (8, 8)
    lat = Lattice(dims)
    U, _ = u1_heatbath(dims, 3.0, 20, 11)
    kd = KDOperator(lat, U, 0.05)
    A = kd.A.toarray()
    Ad = A.conj().T
    E = np.diag(epsilon_dof(lat))
    Binv = kd.Binv.toarray()
    B = kd.B.toarray()
    D = kd.D.toarray()
    assert np.allclose(E @ Ad @ E, Binv @ D, atol=1e-13)
    assert np.allclose(Ad, E @ Binv @ D @ E, atol=1e-13)
    g5L = E @ Binv
    g5R = B @ E
    assert np.allclose(g5L @ A, Ad @ g5L, atol=1e-12)
    assert np.allclose(A @ g5R, g5R @ Ad, atol=1e-13)
    assert np.allclose(g5L @ g5R, np.eye(lat.volume), atol=1e-13)
    # complex-conjugate eigenpairs
    lam = np.linalg.eigvals(A)
    dist = np.abs(np.conj(lam)[:, None] - lam[None, :]).min(axis=1)
    assert dist.max() < 1e-9


def test_block_parity_diagonal_is_identity():
    """A's diagonal blocks are exactly 1 in KD-block parity, not in site parity."""
    dims = (8, 8)
    lat = Lattice(dims)
    U = random_u1(dims, 9)
    kd = KDOperator(lat, U, 0.2)
    A = kd.A.toarray()
    assert np.allclose(A[np.ix_(kd.even, kd.even)], np.eye(kd.even.size), atol=1e-14)
    assert np.allclose(A[np.ix_(kd.odd, kd.odd)], np.eye(kd.odd.size), atol=1e-14)
    se = np.flatnonzero(epsilon_dof(lat) > 0)
    assert not np.allclose(A[np.ix_(se, se)], np.eye(se.size), atol=1e-3)


@pytest.mark.parametrize("nc", [1, 3])
def test_schur_reconstruction_solves_D(nc):
    dims = (8, 8) if nc == 1 else (2, 2, 2, 4)
    lat = Lattice(dims, ncolor=nc)
    U = random_u1(dims, 12) if nc == 1 else random_su3(dims, 12)
    kd = KDOperator(lat, U, 0.1)
    b = gaussian_vectors(1, lat.ndof, 13)[0]
    y_e = np.linalg.solve(kd.S.toarray(), kd.schur_rhs(b))
    x = kd.reconstruct(b, y_e)
    assert np.allclose(x, dense_solve(lat, U, 0.1, b), atol=1e-11)
    # residual identity: b - D x = (b~_e - S y_e, 0) for any y_e
    y_any = gaussian_vectors(1, kd.even.size, 14)[0]
    xa = kd.reconstruct(b, y_any)
    res = b - kd.D @ xa
    assert np.allclose(res[kd.odd], 0, atol=1e-12)
    assert np.allclose(res[kd.even], kd.schur_rhs(b) - kd.S @ y_any, atol=1e-12)


def test_cg_eo_matches_dense():
    dims = (8, 8)
    lat = Lattice(dims)
    U, _ = u1_heatbath(dims, 3.0, 10, 21)
    b = gaussian_vectors(1, lat.ndof, 22)[0]
    x, _ = cg_eo(lat, U, 0.05, b, tol=1e-14)
    assert np.allclose(x, dense_solve(lat, U, 0.05, b), atol=1e-10)


def test_eta_definition():
    lat = Lattice((4, 4, 4, 4))
    c = lat.coords
    assert np.all(eta(lat, 0) == 1)
    assert np.all(eta(lat, 1) == (-1.0) ** c[:, 0])
    assert np.all(eta(lat, 3) == (-1.0) ** (c[:, 0] + c[:, 1] + c[:, 2]))


@pytest.mark.parametrize("bc", [(-1, -1), (-1, 1), (1, 1)])
def test_boundary_signs_per_direction(bc):
    """Boundary signs per direction (the paper is silent; reading of the
    boundary conditions): a sign -1 in direction mu shifts that direction's
    free momenta to (2n + 1) pi / L_mu, so the free spectrum is
    m +- i sqrt(sum sin^2 p) over the shifted zone, and the closed-form FFT
    solve with the matching twist solves D x = b."""
    dims = (8, 12)
    lat = Lattice(dims, bc=bc)
    m = 0.2
    D = dirac_matrix(lat, unit_gauge(dims), m)
    lam = np.linalg.eigvals(D.toarray())
    assert np.allclose(lam.real, m, atol=1e-12)
    # the closed form enumerated here from the momenta, independently of
    # free_spectrum's zone bookkeeping
    ps = [(2 * np.arange(L) + (1 if s == -1 else 0)) * np.pi / L for L, s in zip(dims, bc)]
    g = np.meshgrid(*ps, indexing="ij")
    s2 = np.sort(sum(np.sin(x) ** 2 for x in g).ravel())
    assert np.allclose(np.sort(lam.imag ** 2), s2, atol=1e-11)
    b = gaussian_vectors(1, lat.volume, 7)[0]
    x = free_fft_solve(lat, m, b)
    assert np.linalg.norm(D @ x - b) / np.linalg.norm(b) < 1e-12
    # a hop across the x boundary carries the x sign, across t the t sign
    Dd = D.toarray()
    x0 = lat.index((dims[0] - 1, 3))
    assert np.isclose(Dd[x0, lat.index((0, 3))], 0.5 * bc[0])
    t0 = lat.index((0, dims[1] - 1))
    assert np.isclose(Dd[t0, lat.index((0, 0))], 0.5 * bc[1])


def test_cg_eo_multi_matches_single_and_dense():
    """The block form of the oracle's even/odd CG runs each column's own CG:
    iteration counts within one (summation order moves the stop) and the
    same solutions as cg_eo column by column, and the dense-LU answer."""
    from oracle.exact import cg_eo_multi
    dims = (8, 12)
    lat = Lattice(dims)
    U = random_u1(dims, 4)
    m = 0.15
    B = gaussian_vectors(3, lat.volume, 11)
    X, its = cg_eo_multi(lat, U, m, B, tol=1e-13)
    for q in range(3):
        x1, k1 = cg_eo(lat, U, m, B[q], tol=1e-13)
        assert abs(its[q] - k1) <= 1  # the stop can fall either side by rounding
        assert np.linalg.norm(X[q] - x1) / np.linalg.norm(x1) < 1e-11
        xd = dense_solve(lat, U, m, B[q])
        assert np.linalg.norm(X[q] - xd) / np.linalg.norm(xd) < 1e-10
