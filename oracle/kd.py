"""Oracle: Kahler-Dirac blocking, A = D B^-1 and the block-parity Schur system.

TEST INFRASTRUCTURE ONLY (see oracle/staggered.py).

Sec. 2.1: D = B + C where B is D restricted to the 2^d hypercubes ("Kahler-Dirac
blocks") anchored at even coordinates 2n, mass included, and C holds the hops
between blocks.  The preconditioned operator is A = D B^-1 = 1 + C B^-1
(eq. "defA").  Its adjoint obeys epsilon A^dag epsilon = B^-1 D (eq.
"gamma5L").  The fine solver of Table 1 iterates on the Schur complement
1 - A_eo A_oe, where even/odd is read as the parity of the KD block
(sum_mu floor(x_mu/2) mod 2): only in that parity are A's diagonal blocks the
identity.
"""
import numpy as np
import scipy.sparse as sp

from .staggered import dirac_matrix, dirac_matrix_naik, epsilon_dof


def block_of_site(lat):
    """KD block index of every site (blocks of 2^d sites anchored at 2n)."""
    bdims = np.array(lat.dims) // 2
    bc = lat.coords // 2
    strides = np.cumprod((1,) + tuple(bdims[:-1]))
    return (bc * strides).sum(axis=1)


def block_parity_of_site(lat):
    return (lat.coords // 2).sum(axis=1) % 2


def block_of_dof(lat):
    return np.repeat(block_of_site(lat), lat.ncolor)


def split_B_C(lat, D):
    """B = entries of D inside one KD block (mass included); C = D - B."""
    Dc = D.tocoo()
    blk = block_of_dof(lat)
    inside = blk[Dc.row] == blk[Dc.col]
    n = D.shape[0]
    B = sp.coo_matrix((Dc.data[inside], (Dc.row[inside], Dc.col[inside])),
                      shape=(n, n)).tocsr()
    C = sp.coo_matrix((Dc.data[~inside], (Dc.row[~inside], Dc.col[~inside])),
                      shape=(n, n)).tocsr()
    return B, C


def block_inverse(lat, B):
    """B^-1 by a dense inverse of every KD block, as a sparse matrix."""
    blk = block_of_dof(lat)
    nblk = int(blk.max()) + 1
    bs = (2 ** lat.nd) * lat.ncolor
    order = np.argsort(blk, kind="stable")
    local = np.empty_like(order)
    local[order] = np.arange(order.size) % bs
    Bc = B.tocoo()
    dense = np.zeros((nblk, bs, bs), dtype=np.complex128)
    dense[blk[Bc.row], local[Bc.row], local[Bc.col]] = Bc.data
    inv = np.linalg.inv(dense)
    dofs = order.reshape(nblk, bs)           # dofs of each block, local order
    r = np.repeat(dofs[:, :, None], bs, axis=2).ravel()
    c = np.repeat(dofs[:, None, :], bs, axis=1).ravel()
    n = B.shape[0]
    return sp.coo_matrix((inv.ravel(), (r, c)), shape=(n, n)).tocsr()


class KDOperator:
    """The Kahler-Dirac preconditioned operator A = D B^-1 and its pieces.

    naik=True takes the Naik-improved D (eq. "freehisq").  Its three-link hops
    always leave the KD block, so B is the plain block with its hops scaled by
    9/8 and the new terms sit in C; but a hop from x_mu = 2n + 1 lands two
    blocks away, in a block of the same parity, so A_ee != 1 and the
    block-parity Schur form of the plain operator does not apply (has_schur
    is False; the solver then iterates on the full A)."""

    def __init__(self, lat, U, m, naik=False):
        self.lat = lat
        self.m = float(m)
        self.naik = bool(naik)
        self.D = dirac_matrix_naik(lat, U, m) if naik else dirac_matrix(lat, U, m)
        self.B, self.C = split_B_C(lat, self.D)
        self.Binv = block_inverse(lat, self.B)
        n = self.D.shape[0]
        self.A = (self.D @ self.Binv).tocsr()
        self.Adag = self.A.conj().T.tocsr()
        par = np.repeat(block_parity_of_site(lat), lat.ncolor)
        self.even = np.flatnonzero(par == 0)
        self.odd = np.flatnonzero(par == 1)
        A = self.A
        self.A_eo = A[self.even][:, self.odd].tocsr()
        self.A_oe = A[self.odd][:, self.even].tocsr()
        ne = self.even.size
        self.has_schur = not self.naik
        # Schur complement on even KD blocks (Table 1, level-1 operator)
        self.S = (sp.identity(ne, dtype=np.complex128, format="csr")
                  - self.A_eo @ self.A_oe).tocsr() if self.has_schur else None
        self.eps = epsilon_dof(lat)
        self.n = n

    def schur_rhs(self, b):
        """b~_e = b_e - A_eo b_o."""
        return b[self.even] - self.A_eo @ b[self.odd]

    def reconstruct(self, b, y_e):
        """y_o = b_o - A_oe y_e, then x = B^-1 y (so that D x = b)."""
        y = np.zeros(self.n, dtype=np.complex128)
        y[self.even] = y_e
        y[self.odd] = b[self.odd] - self.A_oe @ y_e
        return self.Binv @ y
