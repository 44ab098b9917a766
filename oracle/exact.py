"""Oracle: exact solutions of D x = b (FP64), the definition the MG solve reaches.

TEST INFRASTRUCTURE ONLY (see oracle/staggered.py).

* ``dense_solve``: LU with partial pivoting (LAPACK through numpy) on the dense
  matrix; small lattices only.
* ``cg_eo``: CG on the site-parity normal equations of Sec. 2 (eq. "normal"):
  (m^2 - D_eo D_oe) x_e = m b_e - D_eo b_o, then x_o = (b_o - D_oe x_e)/m.
  ``cg_eo_multi`` runs the same CG on several right-hand sides at once.
* ``free_fft_solve``: for unit links, D^dag D = m^2 + sum_mu sin^2 p_mu is
  diagonal in momentum space (the corner terms cancel, Sec. 2), so
  x = D^dag F^-1[F(b) / (m^2 + sum sin^2 p)].  Each antiperiodic direction mu
  is handled by the twist exp(i pi x_mu / L_mu), which makes the field periodic.
"""
import numpy as np
import scipy.sparse as sp

from .staggered import dirac_matrix, epsilon
from .mg import cg


def dense_solve(lat, U, m, b):
    D = dirac_matrix(lat, U, m).toarray()
    return np.linalg.solve(D, b)


def cg_eo(lat, U, m, b, tol=1e-13, maxit=200000):
    D = dirac_matrix(lat, U, m)
    par = np.repeat(np.where(epsilon(lat) > 0, 0, 1), lat.ncolor)
    e = np.flatnonzero(par == 0)
    o = np.flatnonzero(par == 1)
    D_eo = D[e][:, o].tocsr()
    D_oe = D[o][:, e].tocsr()
    rhs = m * b[e] - D_eo @ b[o]
    normal = lambda v: m * m * v - D_eo @ (D_oe @ v)
    x_e, its = cg(normal, rhs, tol, maxit)
    x = np.zeros_like(b)
    x[e] = x_e
    x[o] = (b[o] - D_oe @ x_e) / m
    return x, its


def cg_eo_multi(lat, U, m, B, tol=1e-13, maxit=200000):
    """``cg_eo`` for the columns of B [nrhs][ndof] at once: the same CG,
    with its own scalars and its own stop per column, run over a block of
    columns so the sparse products are shared.  Returns (X, iterations)."""
    D = dirac_matrix(lat, U, m)
    par = np.repeat(np.where(epsilon(lat) > 0, 0, 1), lat.ncolor)
    e = np.flatnonzero(par == 0)
    o = np.flatnonzero(par == 1)
    D_eo = D[e][:, o].tocsr()
    D_oe = D[o][:, e].tocsr()
    B = np.asarray(B)
    rhs = (m * B[:, e] - (D_eo @ B[:, o].T).T).T          # [n_e][nrhs]
    x = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    rr = np.einsum("ij,ij->j", r.conj(), r).real
    bnorm = np.sqrt(rr)
    active = bnorm > 0
    its = np.zeros(B.shape[0], dtype=int)
    while active.any() and its.max() < maxit:
        a = np.flatnonzero(active)
        q = m * m * p[:, a] - D_eo @ (D_oe @ p[:, a])
        alpha = rr[a] / np.einsum("ij,ij->j", p[:, a].conj(), q).real
        x[:, a] += alpha * p[:, a]
        r[:, a] -= alpha * q
        its[a] += 1
        rr_new = np.einsum("ij,ij->j", r[:, a].conj(), r[:, a]).real
        done = np.sqrt(rr_new) <= tol * bnorm[a]
        beta = rr_new / rr[a]
        p[:, a] = r[:, a] + beta * p[:, a]
        rr[a] = rr_new
        active[a[done]] = False
    X = np.zeros_like(B)
    X[:, e] = x.T
    X[:, o] = (B[:, o].T - D_oe @ x).T / m
    return X, its


def free_fft_solve(lat, m, b):
    """Closed-form solve for U = 1 (ncolor 1 or more, colours decouple)."""
    nc = lat.ncolor
    shape = tuple(reversed(lat.dims))
    nd = lat.nd
    bb = b.reshape(shape + (nc,))
    twist = np.ones(shape, dtype=np.complex128)
    for mu in range(nd):
        if lat.bc[mu] == -1:
            xm = lat.coords[:, mu].reshape(shape)
            twist = twist * np.exp(1j * np.pi * xm / lat.dims[mu])
    g = bb / twist[..., None]
    ghat = np.fft.fftn(g, axes=tuple(range(nd)))
    denom = np.full(shape, m * m, dtype=np.float64)
    for mu in range(nd):
        L = lat.dims[mu]
        p = 2 * np.pi * np.fft.fftfreq(L) * 1.0
        if lat.bc[mu] == -1:
            p = p + np.pi / L
        sh = [1] * nd
        sh[nd - 1 - mu] = L
        denom = denom + np.sin(p.reshape(sh)) ** 2
    y = np.fft.ifftn(ghat / denom[..., None], axes=tuple(range(nd)))
    y = (y * twist[..., None]).reshape(-1)
    U1 = np.zeros((nd, lat.volume, nc, nc), dtype=np.complex128)
    for a in range(nc):
        U1[:, :, a, a] = 1
    D = dirac_matrix(lat, U1, m)
    return D.conj().T @ y
