"""GPU CG on the site even/odd Schur system (kdmg_solve_cg_eo; the paper's
comparison solver, Sec. 1 and 2) against the oracle's cg_eo.

The oracle runs the same CG recurrence on the same system with the stopping
rule mapped onto its own: the GPU stops a rhs when ||r_e|| <= tol m ||b||,
the oracle when ||r_e|| <= tol' ||rhs_e||, so tol' = tol m ||b|| / ||rhs_e||.
Checked per rhs: iteration counts within one (rounding order differs), true
residual ||b - D x|| / ||b|| <= 1e-10 with the oracle's D, and the solution
within 1e-8 relative of the oracle's.  nrhs 3 and 9 take the hop kernel's
1- and 8-rhs tiles (9: a ragged tail of 1).  The 4D SU(3) form (8^3 x 12,
8 x 4^2 x 12 and 4^3 x 8; 1, 3 and 5 rhs: the 1-, 2- and 4-rhs tiles with
ragged tails) is checked the same way."""
import numpy as np
import pytest

from oracle.staggered import Lattice as OLattice, dirac_matrix, epsilon
from oracle.exact import cg_eo
from synth import u1_heatbath, gaussian_vectors, su3_smooth_random

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_07823_amd import kdmg
    kdmg.kdmg_init(0)
    return kdmg


@pytest.mark.parametrize("dims,beta,m,nrhs", [((16, 32), 3.0, 0.05, 3), ((32, 32), 6.0, 0.02, 9)])
def test_cg_eo_against_oracle(K, dims, beta, m, nrhs):
    U, _ = u1_heatbath(dims, beta, 30, 17)
    olat = OLattice(dims)
    D = dirac_matrix(olat, U, m)
    lat = K.Lattice(dims, U)
    b = gaussian_vectors(nrhs, olat.volume, 81, tag=0)
    x = torch.empty((nrhs, olat.volume), dtype=torch.complex128, device="cuda")
    tol = 1e-10
    its = K.kdmg_solve_cg_eo(lat, m, torch.from_numpy(b).to("cuda"), x, nrhs, tol)
    xs = x.cpu().numpy()
    par = np.where(epsilon(olat) > 0, 0, 1)
    e, o = np.flatnonzero(par == 0), np.flatnonzero(par == 1)
    D_eo = D.tocsr()[e][:, o]
    for r in range(nrhs):
        rhs = m * b[r][e] - D_eo @ b[r][o]
        tol_o = tol * m * np.linalg.norm(b[r]) / np.linalg.norm(rhs)
        xo, its_o = cg_eo(olat, U, m, b[r], tol=tol_o)
        assert abs(its[r] - its_o) <= 1, (r, its[r], its_o)
        assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
        assert np.linalg.norm(xs[r] - xo) / np.linalg.norm(xo) < 1e-8


@pytest.mark.parametrize("dims,m,nrhs", [((8, 8, 8, 12), 0.05, 5), ((8, 4, 4, 12), 0.1, 1),
                                         ((4, 4, 4, 8), 0.02, 3)])
def test_cg_eo_4d_su3_against_oracle(K, dims, m, nrhs):
    U = su3_smooth_random(dims, 0.4, 2, 0.5, 43)
    olat = OLattice(dims, ncolor=3)
    D = dirac_matrix(olat, U, m)
    lat = K.Lattice(dims, U)
    n = olat.ndof
    b = gaussian_vectors(nrhs, n, 82, tag=0)
    x = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
    tol = 1e-10
    its = K.kdmg_solve_cg_eo(lat, m, torch.from_numpy(b).to("cuda"), x, nrhs, tol)
    xs = x.cpu().numpy()
    par = np.repeat(np.where(epsilon(olat) > 0, 0, 1), 3)
    e, o = np.flatnonzero(par == 0), np.flatnonzero(par == 1)
    D_eo = D.tocsr()[e][:, o]
    for r in range(nrhs):
        rhs = m * b[r][e] - D_eo @ b[r][o]
        tol_o = tol * m * np.linalg.norm(b[r]) / np.linalg.norm(rhs)
        xo, its_o = cg_eo(olat, U, m, b[r], tol=tol_o)
        print("4D CG-eo %s rhs %d: %d iterations (oracle %d)" % (dims, r, its[r], its_o))
        assert abs(its[r] - its_o) <= 1, (r, its[r], its_o)
        assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
        assert np.linalg.norm(xs[r] - xo) / np.linalg.norm(xo) < 1e-8


def test_cg_eo_errors(K):
    U, _ = u1_heatbath((16, 16), 3.0, 5, 3)
    lat = K.Lattice((16, 16), U)
    b = torch.zeros((1, 256), dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)
    for kw in (dict(mass=0.0), dict(mass=0.1, tol=0.0), dict(mass=0.1, maxit=0)):
        with pytest.raises(K.KdmgError) as err:
            K.kdmg_solve_cg_eo(lat, kw.pop("mass"), b, x, 1, **kw)
        assert err.value.status == K.KDMG_EINVAL
