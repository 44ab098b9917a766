"""Seeded gauge configurations.

* ``u1_heatbath``: quenched compact U(1) with the Wilson plaquette action
  ``S = beta * sum_P (1 - Re U_P)``, hot start, checkerboard heatbath sweeps.
  For one link with staple sum ``A`` the conditional density of its angle is
  proportional to ``exp(beta |A| cos(theta + arg A))``, a von Mises law, drawn
  with numpy's von Mises sampler.  The paper's ensembles are quenched compact
  U(1) fields at beta = 3, 6, 10 (Sec. 4.1); it does not describe the sampler.
* ``su3_smooth_random``: ``U = exp(i eps H)`` with ``H`` a Gaussian traceless
  Hermitian 3x3 matrix, followed by APE-style smearing with SU(3) projection.

Array layout: angles/links are numpy arrays ``[mu, x_{d-1}, ..., x_1]`` so
that a C-order flatten of the spatial axes gives site index x_1 fastest.
"""
import numpy as np


def config_seed(L, beta, c):
    """Seed of configuration ``c`` of an ``L^d`` lattice at coupling ``beta``."""
    return int(1_000_003 * int(L) + round(101 * float(beta)) + int(c))


def unit_gauge(dims, ncolor=1):
    """Free field: every link the identity.  Returns complex128 [mu, site, a, b]."""
    nd = len(dims)
    V = int(np.prod(dims))
    U = np.zeros((nd, V, ncolor, ncolor), dtype=np.complex128)
    for a in range(ncolor):
        U[:, :, a, a] = 1.0
    return U


def _ax(nd, mu):
    # numpy axis of lattice direction mu in an array shaped [x_{d-1},...,x_1]
    return nd - 1 - mu


def _parity(shape):
    grids = np.indices(shape)
    return (grids.sum(axis=0) & 1)


def u1_heatbath(dims, beta, sweeps, seed):
    """Quenched compact U(1) configuration.

    Returns ``(U, info)`` with ``U`` complex128 [mu, site, 1, 1] and ``info``
    holding the average plaquette and the topological charge of the final
    configuration.
    """
    dims = tuple(int(L) for L in dims)
    nd = len(dims)
    shape = tuple(reversed(dims))
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    theta = rng.uniform(-np.pi, np.pi, size=(nd,) + shape)   # hot start
    par = _parity(shape)
    for _ in range(int(sweeps)):
        for mu in range(nd):
            for p in (0, 1):
                A = np.zeros(shape, dtype=np.complex128)
                for nu in range(nd):
                    if nu == mu:
                        continue
                    am, an = _ax(nd, mu), _ax(nd, nu)
                    # forward staple U_nu(x+mu) U_mu(x+nu)^* U_nu(x)^*
                    fwd = (np.roll(theta[nu], -1, am) - np.roll(theta[mu], -1, an)
                           - theta[nu])
                    # backward staple U_nu(x+mu-nu)^* U_mu(x-nu)^* U_nu(x-nu)
                    t_nu_m = np.roll(theta[nu], 1, an)
                    bwd = (-np.roll(t_nu_m, -1, am) - np.roll(theta[mu], 1, an)
                           + t_nu_m)
                    A += np.exp(1j * fwd) + np.exp(1j * bwd)
                kappa = beta * np.abs(A)
                phi = rng.vonmises(0.0, np.maximum(kappa, 1e-300))
                new = np.angle(np.conj(A)) + phi
                mask = par == p
                theta[mu] = np.where(mask, new, theta[mu])
        theta = np.angle(np.exp(1j * theta))
    U = np.exp(1j * theta).reshape(nd, -1, 1, 1)
    return U, {"plaquette": u1_plaquette(U, dims),
               "topological_charge": _u1_charge(theta, dims)}


def _u1_plaq_angles(theta, dims):
    nd = len(dims)
    out = []
    for mu in range(nd):
        for nu in range(mu + 1, nd):
            am, an = _ax(nd, mu), _ax(nd, nu)
            out.append(theta[mu] + np.roll(theta[nu], -1, am)
                       - np.roll(theta[mu], -1, an) - theta[nu])
    return out


def u1_plaquette(U, dims):
    """Average of Re U_P over all plaquettes."""
    nd = len(dims)
    shape = tuple(reversed(dims))
    theta = np.angle(U.reshape(nd, *shape))
    vals = [np.cos(a).mean() for a in _u1_plaq_angles(theta, dims)]
    return float(np.mean(vals))


def _u1_charge(theta, dims):
    if len(dims) != 2:
        return None
    (a,) = _u1_plaq_angles(theta, dims)
    return float(np.angle(np.exp(1j * a)).sum() / (2 * np.pi))


# ----------------------------------------------------------------- SU(3)

def _gellmann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j; l[1][1, 0] = 1j
    l[2][0, 0] = 1; l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j; l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j; l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3); l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _proj_su3(M):
    """Nearest unitary by polar decomposition, then remove the determinant phase."""
    H = _dag(M) @ M
    w, V = np.linalg.eigh(H)
    inv_sqrt = (V * (1.0 / np.sqrt(w))[..., None, :]) @ _dag(V)
    W = M @ inv_sqrt
    det = np.linalg.det(W)
    return W * np.exp(-1j * np.angle(det) / 3.0)[..., None, None]


def su3_smooth_random(dims, eps, ape_steps, ape_alpha, seed):
    """Smooth random SU(3) field: exp(i eps H) then APE smearing.

    Returns complex128 [mu, site, 3, 3].
    """
    dims = tuple(int(L) for L in dims)
    nd = len(dims)
    shape = tuple(reversed(dims))
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5003]))
    h = rng.standard_normal((nd,) + shape + (8,))
    H = np.einsum("...a,aij->...ij", h, _gellmann() / 2.0)
    w, V = np.linalg.eigh(H)
    U = (V * np.exp(1j * eps * w)[..., None, :]) @ _dag(V)
    for _ in range(int(ape_steps)):
        Unew = np.empty_like(U)
        for mu in range(nd):
            am = _ax(nd, mu)
            stap = np.zeros_like(U[mu])
            for nu in range(nd):
                if nu == mu:
                    continue
                an = _ax(nd, nu)
                Un_xpmu = np.roll(U[nu], -1, am)
                stap += U[nu] @ np.roll(U[mu], -1, an) @ _dag(Un_xpmu)
                Un_xmnu = np.roll(U[nu], 1, an)
                stap += _dag(Un_xmnu) @ np.roll(U[mu], 1, an) @ np.roll(Un_xmnu, -1, am)
            M = (1.0 - ape_alpha) * U[mu] + (ape_alpha / (2 * (nd - 1))) * stap
            Unew[mu] = _proj_su3(M)
        U = Unew
    return U.reshape(nd, -1, 3, 3)


def su3_plaquette(U, dims):
    """Average of Re tr(U_P)/3 over all plaquettes."""
    nd = len(dims)
    shape = tuple(reversed(dims))
    Uf = U.reshape((nd,) + shape + (3, 3))
    vals = []
    for mu in range(nd):
        for nu in range(mu + 1, nd):
            am, an = _ax(nd, mu), _ax(nd, nu)
            P = (Uf[mu] @ np.roll(Uf[nu], -1, am) @ _dag(np.roll(Uf[mu], -1, an))
                 @ _dag(Uf[nu]))
            vals.append(np.trace(P, axis1=-2, axis2=-1).real.mean() / 3.0)
    return float(np.mean(vals))
