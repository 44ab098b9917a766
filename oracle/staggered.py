"""Oracle: the staggered Dirac operator and its symmetries (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library.

Definitions follow the paper's Sec. 1 (eq. "staggeredD") and Sec. 2:

  D_{x,y} = 1/2 sum_mu eta_mu(x) [ U_mu(x) delta_{x+mu,y}
                                  - U_mu(x-mu)^dag delta_{x-mu,y} ] + m delta_{x,y}

with eta_mu(x) = (-1)^{sum_{nu<mu} x_nu} (Sec. 1) and the chirality
epsilon(x) = (-1)^{sum_mu x_mu} (Sec. 2, eq. "epsilon").  Lattice spacing a = 1.
Boundary conditions: the paper is silent.  The default is periodic in every
direction except the last (time), which is antiperiodic, as the workloads
fix it; ``Lattice(bc=...)`` sets a sign per direction (+1 periodic, -1
antiperiodic), carried by every hop that crosses that direction's boundary.

Index conventions: site index x_1 + L_1*(x_2 + L_2*(...)) (x_1 fastest),
dof index site*ncolor + colour.  Gauge fields are complex128 [mu, site, a, b].
"""
import numpy as np
import scipy.sparse as sp


class Lattice:
    """Geometry of a hypercubic torus with a boundary sign per direction."""

    def __init__(self, dims, ncolor=1, antiperiodic_time=True, bc=None):
        self.dims = tuple(int(L) for L in dims)
        self.nd = len(self.dims)
        self.ncolor = int(ncolor)
        self.volume = int(np.prod(self.dims))
        if bc is None:
            bc = [1] * (self.nd - 1) + [-1 if antiperiodic_time else 1]
        self.bc = tuple(int(b) for b in bc)
        assert len(self.bc) == self.nd and all(b in (1, -1) for b in self.bc)
        self.antiperiodic_time = self.bc[-1] == -1
        idx = np.arange(self.volume)
        coords = np.empty((self.volume, self.nd), dtype=np.int64)
        rem = idx.copy()
        for mu, L in enumerate(self.dims):
            coords[:, mu] = rem % L
            rem //= L
        self.coords = coords
        self.strides = np.cumprod((1,) + self.dims[:-1])

    @property
    def ndof(self):
        return self.volume * self.ncolor

    def index(self, coords):
        c = np.asarray(coords) % np.array(self.dims)
        return (c * self.strides).sum(axis=-1)

    def neighbour(self, mu, step):
        """Site index of x + step*mu_hat and the boundary sign of that hop."""
        c = self.coords.copy()
        c[:, mu] += step
        crosses = (c[:, mu] < 0) | (c[:, mu] >= self.dims[mu])
        sign = np.ones(self.volume)
        sign[crosses] = float(self.bc[mu])
        return self.index(c), sign


def eta(lat, mu):
    """Staggered phase eta_mu(x) = (-1)^{sum_{nu<mu} x_nu}  (Sec. 1)."""
    return np.where(lat.coords[:, :mu].sum(axis=1) % 2 == 0, 1.0, -1.0)


def epsilon(lat):
    """Chirality epsilon(x) = (-1)^{sum_mu x_mu}  (Sec. 2, eq. epsilon)."""
    return np.where(lat.coords.sum(axis=1) % 2 == 0, 1.0, -1.0)


def epsilon_dof(lat):
    return np.repeat(epsilon(lat), lat.ncolor)


def dirac_matrix(lat, U, m):
    """Sparse D(U, m) of eq. "staggeredD" as a CSR matrix on dofs."""
    nc = lat.ncolor
    U = np.asarray(U).reshape(lat.nd, lat.volume, nc, nc)
    x = np.arange(lat.volume)
    rows, cols, vals = [], [], []
    for mu in range(lat.nd):
        e = eta(lat, mu)
        fwd, sf = lat.neighbour(mu, +1)
        bwd, sb = lat.neighbour(mu, -1)
        for a in range(nc):
            for b in range(nc):
                # +1/2 eta_mu(x) U_mu(x)_{ab} psi_b(x+mu)
                rows.append(x * nc + a)
                cols.append(fwd * nc + b)
                vals.append(0.5 * e * sf * U[mu, x, a, b])
                # -1/2 eta_mu(x) [U_mu(x-mu)^dag]_{ab} psi_b(x-mu)
                rows.append(x * nc + a)
                cols.append(bwd * nc + b)
                vals.append(-0.5 * e * sb * np.conj(U[mu, bwd, b, a]))
    n = lat.ndof
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(np.full(n, complex(m)))
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                              np.concatenate(cols))),
                      shape=(n, n), dtype=np.complex128)
    return D.tocsr()


# Naik-improved operator (Sec. 2.1, eq. "freehisq").  Printed with an
# overall -1/2 and coefficients 9/16 and 1/48, the operator's own momentum
# symbol would be (1/2) sin p (1 + sin^2 p / 6), half the spectrum printed
# after it; the coefficients that give that spectrum are 9/8 and -1/24 on
# eq. "staggeredD"'s 1/2 hop (and the sign of the hop follows eq.
# "staggeredD", the two conventions being epsilon-similar).  Gauged with the
# product of the three links along the hop.
NAIK_C1 = 9.0 / 8.0
NAIK_C3 = -1.0 / 24.0


def naik_long_links(lat, U):
    """W_mu(x) = U_mu(x) U_mu(x + mu) U_mu(x + 2 mu), the parallel transporter
    of the three-link hop (boundary signs are applied by the operator)."""
    nc = lat.ncolor
    U = np.asarray(U).reshape(lat.nd, lat.volume, nc, nc)
    W = np.empty_like(U)
    for mu in range(lat.nd):
        f1, _ = lat.neighbour(mu, +1)
        f2 = f1[f1]
        W[mu] = U[mu] @ U[mu][f1] @ U[mu][f2]
    return W


def naik_hops(lat, step, mu):
    """Site index of x + step*mu_hat (|step| <= 3 < L_mu) and its boundary sign."""
    c = lat.coords.copy()
    c[:, mu] += step
    crosses = (c[:, mu] < 0) | (c[:, mu] >= lat.dims[mu])
    sign = np.where(crosses, float(lat.bc[mu]), 1.0)
    return lat.index(c), sign


def dirac_matrix_naik(lat, U, m, c1=NAIK_C1, c3=NAIK_C3):
    """Sparse Naik-improved D:
    D = m + 1/2 sum_mu eta_mu(x) [ c1 (U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu))
                                  + c3 (W_mu(x) psi(x+3mu) - W_mu(x-3mu)^dag psi(x-3mu)) ]."""
    nc = lat.ncolor
    U = np.asarray(U).reshape(lat.nd, lat.volume, nc, nc)
    W = naik_long_links(lat, U)
    x = np.arange(lat.volume)
    rows, cols, vals = [], [], []
    for mu in range(lat.nd):
        e = eta(lat, mu)
        for coef, step, L in ((c1, 1, U), (c3, 3, W)):
            fwd, sf = naik_hops(lat, +step, mu)
            bwd, sb = naik_hops(lat, -step, mu)
            for a in range(nc):
                for b in range(nc):
                    rows.append(x * nc + a)
                    cols.append(fwd * nc + b)
                    vals.append(0.5 * coef * e * sf * L[mu, x, a, b])
                    rows.append(x * nc + a)
                    cols.append(bwd * nc + b)
                    vals.append(-0.5 * coef * e * sb * np.conj(L[mu, bwd, b, a]))
    n = lat.ndof
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(np.full(n, complex(m)))
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n), dtype=np.complex128)
    return D.tocsr()


def free_spectrum_naik(lat, m):
    """Closed form of the free Naik spectrum (Sec. 2.1):
    m +- i sqrt(sum_mu sin^2 p_mu (1 + sin^2 p_mu / 6)^2), full zone; returns
    the multiset of (Im lambda)^2 for a single colour."""
    ps = []
    for mu, L in enumerate(lat.dims):
        n = np.arange(L)
        ps.append((2 * n + (1 if lat.bc[mu] == -1 else 0)) * np.pi / L)
    grids = np.meshgrid(*ps, indexing="ij")
    s2 = sum((np.sin(g) * (1 + np.sin(g) ** 2 / 6)) ** 2 for g in grids).ravel()
    return np.sort(s2)


def apply_D(lat, U, m, psi):
    return dirac_matrix(lat, U, m) @ psi


def gauge_rotate(lat, U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag; g is [site, nc, nc].

    No boundary sign enters: the antiperiodic sign is part of D, not of U.
    """
    nc = lat.ncolor
    U = np.asarray(U).reshape(lat.nd, lat.volume, nc, nc)
    out = np.empty_like(U)
    for mu in range(lat.nd):
        fwd, _ = lat.neighbour(mu, +1)
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(g[fwd], -1, -2))
    return out


def gauge_matrix(lat, g):
    """Block-diagonal G with (G psi)(x) = g(x) psi(x)."""
    nc = lat.ncolor
    return sp.block_diag([g[i] for i in range(lat.volume)], format="csr") \
        if nc > 1 else sp.diags(g[:, 0, 0]).tocsr()


def free_spectrum(lat, m):
    """Closed-form free eigenvalues m +- i sqrt(sum_mu sin^2 p_mu) (Sec. 2).

    Enumerates the full Brillouin zone: p_mu = 2 pi n / L_mu in periodic
    directions and (2n + 1) pi / L_mu in antiperiodic ones.
    The full-zone multiset of sum sin^2 p_mu equals the paper's reduced zone
    n in [-L/4+1, L/4] with multiplicity 2^d.  Returns the multiset of
    (Im lambda)^2 values (each appearing once per momentum) for a single colour.
    """
    ps = []
    for mu, L in enumerate(lat.dims):
        n = np.arange(L)
        if lat.bc[mu] == -1:
            ps.append((2 * n + 1) * np.pi / L)
        else:
            ps.append(2 * n * np.pi / L)
    grids = np.meshgrid(*ps, indexing="ij")
    s2 = sum(np.sin(g) ** 2 for g in grids).ravel()
    return np.sort(s2)
