"""Pins of the oracle's asymmetric coarsening (Sec. 5, eqs. prcplx and
thinlu; App. A): chiral doubling with gamma_5^{L/R} and block
bi-orthonormalisation by a thin LU, giving R != P^dag and a coarse operator
with sigma_1^{L/R} Hermiticity, hence exact complex-conjugate eigenpairs."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.staggered import Lattice
from oracle.kd import KDOperator
from oracle.mg import (MGParams, LevelParams, Hierarchy, Solver, asymmetric_transfer, aggregation_level1,
                       lu_nopivot)
from oracle.exact import dense_solve
from synth import u1_heatbath, gaussian_vectors

L = 32


def pair_defect(lam):
    lam = np.asarray(lam)
    return float(max(np.min(np.abs(lam - np.conj(x))) for x in lam))


@pytest.fixture(scope="module")
def field():
    U, _ = u1_heatbath((L, L), 6.0, 200, 11)
    return U


def build(U, m, nlev, asym=True):
    lat = Lattice((L, L))
    levels = [LevelParams((4, 4), 8), LevelParams((2, 2), 8)][:nlev - 1]
    psi0 = [gaussian_vectors(8, lat.volume, 5, tag=1), gaussian_vectors(8, (L // 8) ** 2 * 16, 5, tag=2)]
    return Hierarchy(lat, U, m, MGParams(levels=levels, asymmetric=asym, outer_maxit=200), psi0[:nlev - 1])


def test_thin_lu():
    M = gaussian_vectors(6, 6, 2) + 4 * np.eye(6)
    Lw, Up = lu_nopivot(M)
    assert np.allclose(Lw @ Up, M, atol=1e-13)
    assert np.allclose(np.diag(Lw), 1) and np.allclose(np.triu(Lw, 1), 0) and np.allclose(np.tril(Up, -1), 0)


def test_biorthonormal_and_sigma1_structure(field):
    """R P = 1; the doubled pair obeys P~ sigma_1 = gamma_5^R R~^dag and
    sigma_1 R~ = P~^dag gamma_5^L, so R~ A P~ is sigma_1-Hermitian; after the
    thin LU, sigma_1^L sigma_1^R = 1 and sigma_1^L A_hat = A_hat^dag sigma_1^L."""
    h = build(field, 0.05, 2)
    A = h.kd.A
    P, R = h.P[0], h.R[0]
    nc = P.shape[1]
    assert abs(R @ P - sp.identity(nc)).max() < 1e-12
    gL, gR = h.gamma_pairs[0]
    # gamma_5^{L/R} Hermiticity of the fine operator (eqs. gamma5L, gamma5R)
    assert abs(gL @ A - A.conj().T @ gL).max() < 1e-12
    assert abs(A @ gR - gR @ A.conj().T).max() < 1e-12
    assert abs(gL @ gR - sp.identity(A.shape[0])).max() < 1e-12
    sL, sR = h.gamma_pairs[1]
    Ah = h.ops[1]
    assert abs(sL @ sR - sp.identity(nc)).max() < 1e-10
    assert abs(sL @ Ah - Ah.conj().T @ sL).max() < 1e-8 * abs(Ah).max()
    # sigma_1^L R = P^dag gamma_5^L and P sigma_1^R = gamma_5^R R^dag
    assert abs(sL @ R - P.conj().T @ gL).max() < 1e-9
    assert abs(P @ sR - gR @ R.conj().T).max() < 1e-9


@pytest.mark.parametrize("nlev", [2, 3])
def test_exact_conjugate_pairs(field, nlev):
    """The asymmetric coarse operators keep exact complex-conjugate eigenpairs
    on every level (the symmetric ones only approximately, Sec. 3.3)."""
    h = build(field, 0.05, nlev)
    for lev in range(1, nlev):
        assert pair_defect(np.linalg.eigvals(h.ops[lev].toarray())) < 1e-9
    hs = build(field, 0.05, 2, asym=False)
    assert pair_defect(np.linalg.eigvals(hs.ops[1].toarray())) > 1e-6


def test_exact_eigenpair_preservation(field):
    """Sec. 5: with psi a right eigenvector of A (eigenvalue lambda) and
    psibar the left one, the asymmetric coarse operator has lambda and
    lambda* as exact eigenvalues and P R reproduces both right eigenvectors
    (v and gamma_5^R psibar)."""
    lat = Lattice((16, 16))
    U, _ = u1_heatbath((16, 16), 6.0, 100, 12)
    kd = KDOperator(lat, U, 0.05)
    A = kd.A.toarray()
    lam, Vr = np.linalg.eig(A)
    k = int(np.argmin(np.abs(lam) + 10 * (np.abs(lam.imag) < 1e-6)))  # a complex low mode
    v = Vr[:, k] / np.linalg.norm(Vr[:, k])
    lamL, Wl = np.linalg.eig(A.conj().T)
    w = Wl[:, int(np.argmin(np.abs(lamL - np.conj(lam[k]))))]
    w = w / np.linalg.norm(w)
    E = sp.diags(kd.eps)
    gL, gR = (E @ kd.Binv).tocsr(), (kd.B @ E).tocsr()
    P, R, _, _ = asymmetric_transfer(v[None, :], w[None, :], aggregation_level1(lat, (4, 4)), gL, gR)
    Ah = (R @ kd.A @ P).toarray()
    ch = np.linalg.eigvals(Ah)
    assert np.min(np.abs(ch - lam[k])) < 1e-9 and np.min(np.abs(ch - np.conj(lam[k]))) < 1e-9
    vm = gR @ w
    assert np.linalg.norm(A @ vm - np.conj(lam[k]) * vm) < 1e-9 * np.linalg.norm(vm)
    for u in (v, vm):
        assert np.linalg.norm(P @ (R @ u) - u) < 1e-9 * np.linalg.norm(u)


def test_asymmetric_solve(field):
    """Two levels with the asymmetric coarsening solve to 1e-10 and the
    dense-LU answer (measured: 16 outer iterations at m = 0.05, as the
    symmetric coarsening's 15).  With three levels the recursive form is far
    weaker here (140 outer iterations at m = 0.05, no convergence within 200
    at m = 0.01), as App. A reports for two dimensions."""
    h = build(field, 0.05, 2)
    b = gaussian_vectors(1, L * L, 6)[0]
    x, info = Solver(h).solve(b, 1e-10)
    assert info["converged"] and info["outer_its"] <= 30, info
    xd = dense_solve(h.lat, field, 0.05, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8


def test_asymmetric_coarse_operator_conditioning():
    """App. A finds the asymmetric form less stable in two dimensions.  On a
    smooth 32^2 field (beta = 10, m = 0.001, 4x4 aggregates, n_vec 16) its
    coarse operator is about a hundred times worse conditioned than the
    symmetric one (measured 3.7e4 against 390), which is what defeats the
    coarsest CGNE(0.2) there."""
    from synth import config_seed
    seed = config_seed(32, 10.0, 0)
    U, _ = u1_heatbath((32, 32), 10.0, 200, seed)
    lat = Lattice((32, 32))
    psi0 = [gaussian_vectors(16, lat.volume, seed, tag=1)]
    conds = []
    for asym in (False, True):
        h = Hierarchy(lat, U, 0.001, MGParams(levels=[LevelParams((4, 4), 16)], asymmetric=asym), psi0)
        s = np.linalg.svd(h.ops[1].toarray(), compute_uv=False)
        conds.append(s[0] / s[-1])
    assert conds[1] > 30 * conds[0], conds
