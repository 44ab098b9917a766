"""Oracle: exact solutions of D x = b (FP64), the definition the MG solve reaches.

TEST INFRASTRUCTURE ONLY (see oracle/staggered.py).

* ``dense_solve``: LU with partial pivoting (LAPACK through numpy) on the dense
  matrix; small lattices only.
* ``cg_eo``: CG on the site-parity normal equations of Sec. 2 (eq. "normal"):
  (m^2 - D_eo D_oe) x_e = m b_e - D_eo b_o, then x_o = (b_o - D_oe x_e)/m.
* ``free_fft_solve``: for unit links, D^dag D = m^2 + sum_mu sin^2 p_mu is
  diagonal in momentum space (the corner terms cancel, Sec. 2), so
  x = D^dag F^-1[F(b) / (m^2 + sum sin^2 p)].  The antiperiodic time direction
  is handled by the twist exp(i pi t / L_t), which makes the field periodic.
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


def free_fft_solve(lat, m, b):
    """Closed-form solve for U = 1 (ncolor 1 or more, colours decouple)."""
    nc = lat.ncolor
    shape = tuple(reversed(lat.dims))
    nd = lat.nd
    bb = b.reshape(shape + (nc,))
    t = lat.coords[:, nd - 1].reshape(shape)
    twist = np.exp(1j * np.pi * t / lat.dims[-1]) if lat.antiperiodic_time \
        else np.ones(shape)
    g = bb / twist[..., None]
    ghat = np.fft.fftn(g, axes=tuple(range(nd)))
    denom = np.full(shape, m * m, dtype=np.float64)
    for mu in range(nd):
        L = lat.dims[mu]
        p = 2 * np.pi * np.fft.fftfreq(L) * 1.0
        if lat.antiperiodic_time and mu == nd - 1:
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
