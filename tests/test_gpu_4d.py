"""GPU parity for the 4D SU(3) staggered operator and its KD multigrid
(eq. "staggeredD" with d = 4, N_c = 3; Sec. 2.1 blocking; Sec. 3 and 4), on
8^4 lattices with smooth random SU(3) fields, against the FP64 oracle.

Tolerances: FP64 operators <= 1e-12 relative max-norm (the dense 48 x 48
block inverse, by Gauss-Jordan on the Hermitian positive Schur forms, adds
rounding of order cond * eps: <= 1e-11 at m >= 0.1); FP16-link D and FP16-P
transfers element by element within 2^-11 (plus FP32 accumulation) times the
sum of the absolute terms (tests/mixed_bounds.py); P and A_hat from identical (unrelaxed) vectors <= 1e-10
(Cholesky-QR applied twice against Householder QR); solves: true residual
<= 1e-10 and ||x - x_cg|| / ||x_cg|| <= 1e-8 against the oracle's CG on the
even/odd normal equations (tolerance 1e-13).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle.staggered import Lattice as OLattice, dirac_matrix
from oracle.kd import KDOperator
from oracle.mg import MGParams, LevelParams, Hierarchy as OHierarchy
from oracle.exact import cg_eo
from mixed_bounds import fp16_coef, abs_terms, rounded, check_elementwise
from synth import su3_smooth_random, gaussian_vectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIMS = (8, 8, 8, 8)


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_07823_amd import kdmg
    kdmg.kdmg_init(0)
    return kdmg


@pytest.fixture(scope="module")
def field():
    return su3_smooth_random(DIMS, 0.4, 2, 0.5, 41)


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("nrhs", [1, 3, 5, 11])
def test_apply_D_4d(K, field, nrhs):
    olat = OLattice(DIMS, ncolor=3)
    m = 0.1
    D = dirac_matrix(olat, field, m)
    lat = K.Lattice(DIMS, field)
    v = gaussian_vectors(nrhs, olat.ndof, 3, tag=0)
    out = torch.empty((nrhs, olat.ndof), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v), out, nrhs)
    ref = (D @ v.T).T
    assert relerr(out.cpu().numpy(), ref) < 1e-12
    out32 = torch.empty((nrhs, olat.ndof), dtype=torch.complex64, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v, torch.complex64), out32, nrhs, prec=K.KDMG_MIXED)
    v32 = rounded(v)
    check_elementwise(out32.cpu().numpy(), (D @ v32.T).T, abs_terms(D, v32), fp16_coef(25), "4D D mixed")


@pytest.mark.parametrize("m,nr", [(0.1, 2), (0.5, 2), (0.1, 5), (0.1, 11)])
def test_fine_operators_4d(K, field, m, nr):
    """nr = 5 takes the hop kernel's 4-rhs tile with a ragged tail; nr = 11 the
    8-rhs tile of the FP32 hop (apply_D mixed) and the 4-rhs FP64 tiles."""
    olat = OLattice(DIMS, ncolor=3)
    kd = KDOperator(olat, field, m)
    lat = K.Lattice(DIMS, field)
    v = gaussian_vectors(nr, olat.ndof, 4, tag=0)
    out = torch.empty((nr, olat.ndof), dtype=torch.complex128, device="cuda")
    for fn, ref in ((lambda o: K.kdmg_apply_A(lat, m, dev(v), o, nr), kd.A),
                    (lambda o: K.kdmg_apply_A(lat, m, dev(v), o, nr, dagger=True), kd.Adag),
                    (lambda o: K.kdmg_apply_Binv(lat, m, dev(v), o, nr), kd.Binv)):
        fn(out)
        assert relerr(out.cpu().numpy(), (ref @ v.T).T) < 1e-11
    ve = v[:, :olat.ndof // 2]
    oute = torch.empty((nr, olat.ndof // 2), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_schur(lat, m, dev(ve), oute, nr)
    assert relerr(oute.cpu().numpy(), (kd.S @ ve.T).T) < 1e-11


def oracle_relaxed(dims, U, m, levels, seed):
    olat = OLattice(dims, ncolor=3)
    psi = []
    n = olat.ndof
    nsites = olat.volume // 16
    for k, (agg, nv) in enumerate(levels):
        psi.append(gaussian_vectors(nv, n, seed, tag=1 + k))
        nsites //= int(np.prod(agg))
        n = nsites * 2 * nv
    params = MGParams(levels=[LevelParams(a, nv) for a, nv in levels])
    return OHierarchy(olat, U, m, params, [("relaxed", V) for V in psi]), psi


def assemble4(op, dims):
    """Stencil blocks [dir][Z][i][j] of a 4D coarse lattice -> dense matrix."""
    ndir, ns, nd, _ = op.shape
    M = np.zeros((ns * nd, ns * nd), dtype=np.complex128)
    for Z in range(ns):
        c, r = [], Z
        for L in dims:
            c.append(r % L)
            r //= L

        def idx(cc):
            s, st = 0, 1
            for x, L in zip(cc, dims):
                s += (x % L) * st
                st *= L
            return s
        nbrs = [Z]
        for mu in range(4):
            for sg in (1, -1):
                cc = list(c)
                cc[mu] += sg
                nbrs.append(idx(cc))
        for d in range(ndir):
            M[Z * nd:(Z + 1) * nd, nbrs[d] * nd:(nbrs[d] + 1) * nd] += op[d, Z]
    return M


def oracle_P_values(h, k):
    P = h.P[k].tocsr()
    ag = h.aggr[k]
    nv = h.params.levels[k].nvec
    rows = np.arange(P.shape[0])
    out = np.zeros((P.shape[0], nv), dtype=np.complex128)
    for i in range(nv):
        cols = ag.agg_of_dof * 2 * nv + ag.chir_of_dof * nv + i
        out[:, i] = np.asarray(P[rows, cols]).ravel()
    return out


def test_hierarchy_4d_from_given_vectors(K, field):
    """P (thin QR per aggregate-chirality) and A_hat = P^dag A P from the same
    vectors: GPU Cholesky-QR2 and 4D Galerkin kernels against the oracle."""
    m = 0.1
    levels = [((2, 2, 2, 2), 8)]
    oh, psi = oracle_relaxed(DIMS, field, m, levels, 51)
    lat = K.Lattice(DIMS, field)
    gh = K.Hierarchy(lat, m, K.make_params(levels), psi, relaxed=True)
    assert relerr(gh.prolongator_values(0), oracle_P_values(oh, 0)) < 1e-10
    dims_c, _ = gh.level_info(1)
    assert dims_c == (2, 2, 2, 2)
    Ag = assemble4(gh.coarse_op(1), dims_c)
    assert relerr(Ag, oh.ops[1].toarray()) < 1e-10
    # level-0 transfers with 5 and 11 rhs (rhs tiles of 4 and 8 with ragged
    # tails): FP64 against the oracle's P to 1e-10 (P itself agrees to that
    # given the same vectors); the FP16-P mixed form element by element
    # within 2^-11 (plus FP32 accumulation) times the sum of absolute terms,
    # widened by the 1e-10 the two P's may differ by
    P = oh.P[0]
    Ph = P.conj().T.tocsr()
    nf, nc = P.shape
    ntr, ntp = int(np.diff(Ph.indptr).max()), int(np.diff(P.tocsr().indptr).max())
    for nr, prec, dt in ((5, K.KDMG_FP64, torch.complex128), (5, K.KDMG_MIXED, torch.complex64),
                         (11, K.KDMG_FP64, torch.complex128), (11, K.KDMG_MIXED, torch.complex64)):
        v = gaussian_vectors(nr, nf, 55, tag=0)
        e = gaussian_vectors(nr, nc, 56, tag=0)
        rc = torch.empty((nr, nc), dtype=dt, device="cuda")
        K.kdmg_restrict(gh, 0, dev(v, dt), rc, nr, prec=prec)
        pf = torch.empty((nr, nf), dtype=dt, device="cuda")
        K.kdmg_prolong(gh, 0, dev(e, dt), pf, nr, prec=prec)
        if prec == K.KDMG_FP64:
            assert relerr(rc.cpu().numpy(), (Ph @ v.T).T) < 1e-10
            assert relerr(pf.cpu().numpy(), (P @ e.T).T) < 1e-10
        else:
            v32, e32 = rounded(v), rounded(e)
            check_elementwise(rc.cpu().numpy(), (Ph @ v32.T).T, abs_terms(Ph, v32), fp16_coef(ntr) + 1e-10,
                              "4D restrict mixed")
            check_elementwise(pf.cpu().numpy(), (P @ e32.T).T, abs_terms(P, e32), fp16_coef(ntp) + 1e-10,
                              "4D prolong mixed")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_level_solve_4d(K, field, prec):
    m = 0.1
    levels = [((2, 2, 2, 2), 12)]
    olat = OLattice(DIMS, ncolor=3)
    lat = K.Lattice(DIMS, field)
    n = olat.ndof
    psi = [gaussian_vectors(12, n, 61, tag=1)]
    gh = K.Hierarchy(lat, m, K.make_params(levels, coarse_maxit=1024), psi)
    b = gaussian_vectors(2, n, 62, tag=0)
    x = torch.empty((2, n), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, 2, 1e-10, prec=p)
    D = dirac_matrix(olat, field, m)
    xs = x.cpu().numpy()
    for r in range(2):
        assert info[r]["converged"]
        assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
        xc, _ = cg_eo(olat, field, m, b[r])
        assert np.linalg.norm(xs[r] - xc) / np.linalg.norm(xc) < 1e-8


def test_hierarchy_at_mass_4d(K, field):
    """kdmg_hierarchy_at_mass on a 4D lattice rebuilds B^-1 and A_hat at the
    new mass from the same prolongators: equal to the oracle's hierarchy from
    the same vectors at that mass; the derived hierarchy solves to 1e-10."""
    m0, m1 = 0.1, 0.3
    levels = [((2, 2, 2, 2), 8)]
    oh1, psi = oracle_relaxed(DIMS, field, m1, levels, 52)
    lat = K.Lattice(DIMS, field)
    base = K.Hierarchy(lat, m0, K.make_params(levels), psi, relaxed=True)
    h = base.at_mass(m1)
    dims_c, _ = h.level_info(1)
    assert relerr(assemble4(h.coarse_op(1), dims_c), oh1.ops[1].toarray()) < 1e-10
    olat = OLattice(DIMS, ncolor=3)
    b = gaussian_vectors(1, olat.ndof, 63, tag=0)
    x = torch.empty((1, olat.ndof), dtype=torch.complex128, device="cuda")
    info, _ = K.kdmg_solve(h, dev(b), x, 1, 1e-10, prec=K.KDMG_MIXED)
    D = dirac_matrix(olat, field, m1)
    assert info[0]["converged"]
    assert np.linalg.norm(b[0] - D @ x.cpu().numpy()[0]) / np.linalg.norm(b[0]) <= 1e-10


def test_exact_coarsest_4d(K, field):
    """The exact coarsest solve (coarse_solver = 1) on a 4D SU(3) hierarchy,
    whose coarse stencil has nine directions (the site and +-mu, mu = 0..3):
    the GPU's explicit inverse, built from the same vectors as the oracle's
    coarse operator (the two operators agree to 1e-10), solves that operator
    to 1e-9 against its dense LU for 5 rhs (a ragged 16-rhs tile), and the
    FP64 and mixed KD-MG solves with it reach 1e-10 and agree with the
    oracle's CG-eo to 1e-8."""
    m = 0.1
    levels = [((2, 2, 2, 2), 8)]
    oh, psi = oracle_relaxed(DIMS, field, m, levels, 54)
    lat = K.Lattice(DIMS, field)
    gh = K.Hierarchy(lat, m, K.make_params(levels, coarse_solver=1), psi, relaxed=True)
    A = oh.ops[1].toarray()
    n = A.shape[0]
    assert gh.ndof(1) == n
    r = gaussian_vectors(5, n, 57, tag=0)
    out = torch.empty((5, n), dtype=torch.complex128, device="cuda")
    K.kdmg_coarsest_solve(gh, dev(r), out, 5)
    xg = out.cpu().numpy()
    lu = scipy.linalg.lu_factor(A)
    for q in range(5):
        xo = scipy.linalg.lu_solve(lu, r[q])
        assert np.linalg.norm(xg[q] - xo) / np.linalg.norm(xo) <= 1e-9, q
    olat = OLattice(DIMS, ncolor=3)
    D = dirac_matrix(olat, field, m)
    b = gaussian_vectors(2, olat.ndof, 58, tag=0)
    xc = [cg_eo(olat, field, m, b[q])[0] for q in range(2)]
    for p in (K.KDMG_FP64, K.KDMG_MIXED):
        x = torch.empty((2, olat.ndof), dtype=torch.complex128, device="cuda")
        info, _ = K.kdmg_solve(gh, dev(b), x, 2, 1e-10, prec=p)
        xs = x.cpu().numpy()
        for q in range(2):
            assert info[q]["converged"], (p, q)
            assert np.linalg.norm(b[q] - D @ xs[q]) / np.linalg.norm(b[q]) <= 1e-10
            assert np.linalg.norm(xs[q] - xc[q]) / np.linalg.norm(xc[q]) < 1e-8
