"""Oracle: spectral diagnostics of a Galerkin coarsening (Sec. 3.2, 3.3).

TEST INFRASTRUCTURE ONLY (see oracle/staggered.py).

For a fine operator M (the staggered D, or the KD-preconditioned A), a
prolongator P and a restrictor R (R = P^dag for the symmetric coarsening):
  * local co-linearity of an eigenvector v: ||(1 - P R) v||, how much of v
    the coarse space misses;
  * the oblique (Petrov-Galerkin) projector P_ob = 1 - P (R M P)^-1 R M,
    which maps the error before an exact coarse correction to the error
    after it; ||P_ob v|| below 1 reduces that component, above 1 enhances it;
  * the spectrum of the coarse operator R M P.
Dense linear algebra: lattices of a few thousand dofs at most.
"""
import numpy as np


def eigs_by_magnitude(M):
    """Eigenvalues and unit right eigenvectors of a (small) operator, sorted by |lambda|."""
    A = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    lam, V = np.linalg.eig(A)
    order = np.argsort(np.abs(lam), kind="stable")
    lam, V = lam[order], V[:, order]
    return lam, V / np.linalg.norm(V, axis=0)


def coarse_projector(P, R):
    """PR as a dense matrix."""
    P = P.toarray() if hasattr(P, "toarray") else np.asarray(P)
    R = R.toarray() if hasattr(R, "toarray") else np.asarray(R)
    return P @ R


def oblique_projector(P, R, M):
    """1 - P (R M P)^-1 R M."""
    P = P.toarray() if hasattr(P, "toarray") else np.asarray(P)
    R = R.toarray() if hasattr(R, "toarray") else np.asarray(R)
    A = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    RM = R @ A
    return np.eye(A.shape[0]) - P @ np.linalg.solve(RM @ P, RM)


def colinearity(P, R, V):
    """||(1 - P R) v|| for every column v of V."""
    PR = coarse_projector(P, R)
    return np.linalg.norm(V - PR @ V, axis=0)


def oblique_action(P, R, M, V):
    """||P_ob v|| for every column v of V."""
    return np.linalg.norm(oblique_projector(P, R, M) @ V, axis=0)


def coarse_spectrum(P, R, M):
    """Eigenvalues of R M P."""
    P = P.toarray() if hasattr(P, "toarray") else np.asarray(P)
    R = R.toarray() if hasattr(R, "toarray") else np.asarray(R)
    A = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    return np.linalg.eigvals(R @ A @ P)
