"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical seeded inputs.  Tolerances:
  * FP64 kernels: relative max-norm error <= 1e-12 (rounding order only);
  * FP16-link / FP16-P / FP32 kernels: element by element against the oracle
    applied to the same FP32-rounded input, |err_i| <= c T_i with T_i the sum
    of the absolute values of output i's terms and c = 2^-11 (the relative
    rounding of an FP16-stored complex value) plus the FP32 accumulation bound
    (tests/mixed_bounds.py); FP32-stored coarse operators with c from FP32
    rounding and accumulation alone;
  * solves: true residual <= 1e-10 and ||x - x_oracle|| / ||x_oracle|| <= 1e-8.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.staggered import Lattice as OLattice, dirac_matrix
from oracle.kd import KDOperator
from oracle.mg import MGParams, LevelParams, Hierarchy as OHierarchy, Solver as OSolver
from oracle.exact import dense_solve
from synth import u1_heatbath, gaussian_vectors, unit_gauge
from mixed_bounds import fp16_coef, fp32_coef, abs_terms, rounded, check_elementwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_07823_amd import kdmg
    kdmg.kdmg_init(0)
    return kdmg


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [((16, 16), 3.0, 0.1), ((24, 20), 6.0, 0.01), ((8, 12), 3.0, 0.5)]


def field(dims, beta, seed=7, sweeps=30):
    U, _ = u1_heatbath(dims, beta, sweeps, seed)
    return U


@pytest.mark.parametrize("dims,beta,m", CASES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_apply_D_fp64(K, dims, beta, m, nrhs):
    U = field(dims, beta)
    lat = K.Lattice(dims, U)
    V = lat.volume
    v = gaussian_vectors(nrhs, V, 11)
    out = torch.empty((nrhs, V), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v), out, nrhs)
    torch.cuda.synchronize()
    D = dirac_matrix(OLattice(dims), U, m)
    ref = (D @ v.T).T
    assert relerr(out.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("dims,beta,m", CASES[:2])
def test_apply_D_mixed(K, dims, beta, m):
    U = field(dims, beta)
    lat = K.Lattice(dims, U)
    V = lat.volume
    nrhs = 4
    v = gaussian_vectors(nrhs, V, 12)
    out = torch.empty((nrhs, V), dtype=torch.complex64, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v, torch.complex64), out, nrhs, prec=K.KDMG_MIXED)
    torch.cuda.synchronize()
    D = dirac_matrix(OLattice(dims), U, m)
    v32 = rounded(v)
    check_elementwise(out.cpu().numpy(), (D @ v32.T).T, abs_terms(D, v32), fp16_coef(5), "D mixed")


@pytest.mark.parametrize("dims,beta,m", CASES)
def test_apply_A_mixed(K, dims, beta, m):
    """kdmg_apply_A in the mixed form (FP16 links, B^-1 recomputed in FP32
    from them, FP32 vectors): A = 1 + C B^-1 and A^dag = 1 + eps B^-1 C eps
    element by element.  The FP16 links perturb B by dB, |dB| <= 2^-11 |K|
    (K = B - m), so B^-1 v moves by at most |B^-1| |dB| |B^-1| |v| to first
    order, and C's own rounding adds 2^-11 |C| |B^-1 v|:
      |err| <= 1.25 * 2^-11 (|C| |B^-1| |K| |B^-1| |v| + |C| |B^-1| |v|)
               + FP32 rounding of the same terms."""
    U = field(dims, beta)
    lat = K.Lattice(dims, U)
    kd = KDOperator(OLattice(dims), U, m)
    V = lat.volume
    nrhs = 3
    v32 = rounded(gaussian_vectors(nrhs, V, 15))
    Kb = (kd.B - m * sp.identity(V)).tocsr()
    aB, aC, aK = abs(kd.Binv), abs(kd.C), abs(Kb)
    av = np.abs(v32).T
    t_a = aC @ (aB @ (aK @ (aB @ av))) + aC @ (aB @ av)
    t_d = aB @ (aK @ (aB @ (aC @ av))) + aB @ (aC @ av)
    for dag, ref, t in ((False, kd.A, t_a), (True, kd.Adag, t_d)):
        out = torch.empty((nrhs, V), dtype=torch.complex64, device="cuda")
        K.kdmg_apply_A(lat, m, dev(v32, torch.complex64), out, nrhs, dagger=dag, prec=K.KDMG_MIXED)
        torch.cuda.synchronize()
        bound = 1.25 * 2.0 ** -11 * t.T + fp32_coef(64) * (t.T + np.abs(v32))
        err = np.abs(out.cpu().numpy().astype(np.complex128) - (ref @ v32.T).T)
        assert float(np.max(err / bound)) <= 1.0, (dag, float(np.max(err / bound)))


@pytest.mark.parametrize("nrhs", [5, 11])
def test_apply_D_rhs_tiles(K, nrhs):
    """128^2 (large enough for several rhs per thread): 5 rhs take the 4-rhs
    tile with a ragged tail, 11 the 8-rhs tile with a ragged tail; FP64 to
    1e-12 and mixed element-wise within the FP16-link bound."""
    dims, beta, m = (128, 128), 6.0, 0.01
    U = field(dims, beta)
    lat = K.Lattice(dims, U)
    V = lat.volume
    v = gaussian_vectors(nrhs, V, 13)
    ref = (dirac_matrix(OLattice(dims), U, m) @ v.T).T
    out = torch.empty((nrhs, V), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v), out, nrhs)
    torch.cuda.synchronize()
    assert relerr(out.cpu().numpy(), ref) < 1e-12
    out32 = torch.empty((nrhs, V), dtype=torch.complex64, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v, torch.complex64), out32, nrhs, prec=K.KDMG_MIXED)
    torch.cuda.synchronize()
    D = dirac_matrix(OLattice(dims), U, m)
    v32 = rounded(v)
    check_elementwise(out32.cpu().numpy(), (D @ v32.T).T, abs_terms(D, v32), fp16_coef(5), "D mixed tiles")


@pytest.mark.parametrize("dims,beta,m", CASES)
def test_fine_operators_fp64(K, dims, beta, m):
    U = field(dims, beta)
    lat = K.Lattice(dims, U)
    kd = KDOperator(OLattice(dims), U, m)
    V = lat.volume
    nrhs = 2
    v = gaussian_vectors(nrhs, V, 13)
    for fn, ref in ((lambda i, o: K.kdmg_apply_A(lat, m, i, o, nrhs), kd.A),
                    (lambda i, o: K.kdmg_apply_A(lat, m, i, o, nrhs, dagger=True), kd.Adag),
                    (lambda i, o: K.kdmg_apply_Binv(lat, m, i, o, nrhs), kd.Binv)):
        out = torch.empty((nrhs, V), dtype=torch.complex128, device="cuda")
        fn(dev(v), out)
        torch.cuda.synchronize()
        assert relerr(out.cpu().numpy(), (ref @ v.T).T) < 1e-12
    ve = gaussian_vectors(nrhs, V // 2, 14)
    out = torch.empty((nrhs, V // 2), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_schur(lat, m, dev(ve), out, nrhs)
    torch.cuda.synchronize()
    assert relerr(out.cpu().numpy(), (kd.S @ ve.T).T) < 1e-12


def oracle_setup(dims, U, m, levels, seed):
    olat = OLattice(dims)
    params = MGParams(levels=[LevelParams(a, nv) for a, nv in levels])
    psi0 = []
    n = olat.ndof
    ncs = None
    for k, (agg, nv) in enumerate(levels):
        psi0.append(gaussian_vectors(nv, n, seed, tag=1 + k))
        if k == 0:
            ncs = olat.volume // int(np.prod([2 * a for a in agg]))
        else:
            ncs = ncs // int(np.prod(agg))
        n = ncs * 2 * nv
    return OHierarchy(olat, U, m, params, psi0), psi0


def gpu_params(K, levels, **kw):
    return K.make_params(levels, **kw)


def assemble(op, dims):
    """GPU stencil blocks [dir][Z][i][j] -> dense matrix (coinciding neighbours add)."""
    ndir, ns, nd, _ = op.shape
    M = np.zeros((ns * nd, ns * nd), dtype=np.complex128)
    L0, L1 = dims
    for Z in range(ns):
        z0, z1 = Z % L0, Z // L0
        nbrs = [Z, (z0 + 1) % L0 + L0 * z1, (z0 - 1) % L0 + L0 * z1,
                z0 + L0 * ((z1 + 1) % L1), z0 + L0 * ((z1 - 1) % L1)]
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


H_CASES = [((16, 16), 3.0, 0.1, [((4, 4), 8)]),
           ((32, 32), 6.0, 0.02, [((2, 2), 8), ((2, 2), 8)]),
           ((24, 40), 3.0, 0.05, [((3, 5), 8)])]


@pytest.mark.parametrize("dims,beta,m,levels", H_CASES)
def test_hierarchy_from_relaxed_vectors(K, dims, beta, m, levels):
    """Given the oracle's relaxed null vectors, the GPU's P and coarse operators
    match the oracle's to rounding."""
    U = field(dims, beta)
    oh, _ = oracle_setup(dims, U, m, levels, 21)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), oh.nullvecs, relaxed=True)
    for k in range(len(levels)):
        Pg = gh.prolongator_values(k)
        assert relerr(Pg, oracle_P_values(oh, k)) < 1e-11
        dims_c, _ = gh.level_info(k + 1)
        Ag = assemble(gh.coarse_op(k + 1), dims_c)
        Ao = oh.ops[k + 1].toarray()
        assert relerr(Ag, Ao) < 1e-11


RELAX_CASES = [((16, 16), 3.0, 0.5, [((4, 4), 8)], 1e-9),
               ((16, 16), 3.0, 0.1, [((4, 4), 8)], 1e-2),
               ((32, 32), 6.0, 0.02, [((2, 2), 8), ((2, 2), 8)], 1e-2)]


@pytest.mark.parametrize("dims,beta,m,levels,bound", RELAX_CASES)
def test_hierarchy_relaxation_matches_oracle(K, dims, beta, m, levels, bound):
    """GPU CG relaxation from the same Gaussian starts.  Both sides stop CG at
    ||A A^dag psi|| <= 1e-4 ||A A^dag psi0|| (or 250 iterations); rounding-order
    differences change the iterate by up to the tolerance-sized remainder, so
    the vectors agree to 1e-9 where CG converges in few iterations (m = 0.5)
    and to 1e-2 otherwise, and every GPU vector meets the stopping rule."""
    U = field(dims, beta)
    oh, psi0 = oracle_setup(dims, U, m, levels, 22)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), psi0)
    v0 = gh.nullvecs(0)
    assert np.linalg.norm(v0 - oh.nullvecs[0]) / np.linalg.norm(oh.nullvecs[0]) < bound
    A = oh.kd.A
    for v, s, its in zip(v0, psi0[0], oh.setup_its[0]):
        nrm = lambda u: np.linalg.norm(A @ (A.conj().T @ u))
        if its < 250:
            assert nrm(v) <= 1.0001e-4 * nrm(s)


@pytest.mark.parametrize("dims,beta,m,levels", H_CASES[1:2])
def test_transfer_and_coarse_apply(K, dims, beta, m, levels):
    U = field(dims, beta)
    oh, _ = oracle_setup(dims, U, m, levels, 23)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), oh.nullvecs, relaxed=True)
    # rhs counts: one, a ragged tail of the 8-rhs prolongation tile and of the
    # 32-rhs restriction tile.  FP64 to 1e-12; the mixed form (FP16-stored P,
    # FP32 vectors and arithmetic) element-wise within 2^-11 (plus FP32
    # accumulation) times the sum of the absolute terms
    nrhs = 3
    for k in range(len(levels)):
        nf = gh.ndof(k)
        nc = gh.ndof(k + 1)
        P = oh.P[k]
        for nr in (1, nrhs, 37):
            v = gaussian_vectors(nr, nf, 30 + k + nr)
            ref = (P.conj().T @ v.T).T
            out = torch.empty((nr, nc), dtype=torch.complex128, device="cuda")
            K.kdmg_restrict(gh, k, dev(v), out, nr)
            torch.cuda.synchronize()
            assert relerr(out.cpu().numpy(), ref) < 1e-12
            out32 = torch.empty((nr, nc), dtype=torch.complex64, device="cuda")
            K.kdmg_restrict(gh, k, dev(v, torch.complex64), out32, nr, prec=K.KDMG_MIXED)
            torch.cuda.synchronize()
            v32 = rounded(v)
            Ph = P.conj().T
            nt = int(np.diff(Ph.tocsr().indptr).max())
            check_elementwise(out32.cpu().numpy(), (Ph @ v32.T).T, abs_terms(Ph, v32), fp16_coef(nt),
                              "restrict mixed k=%d nrhs=%d" % (k, nr))
            e = gaussian_vectors(nr, nc, 40 + k + nr)
            ref = (P @ e.T).T
            outp = torch.empty((nr, nf), dtype=torch.complex128, device="cuda")
            K.kdmg_prolong(gh, k, dev(e), outp, nr)
            torch.cuda.synchronize()
            assert relerr(outp.cpu().numpy(), ref) < 1e-12
            outp32 = torch.empty((nr, nf), dtype=torch.complex64, device="cuda")
            K.kdmg_prolong(gh, k, dev(e, torch.complex64), outp32, nr, prec=K.KDMG_MIXED)
            torch.cuda.synchronize()
            e32 = rounded(e)
            nt = int(np.diff(P.tocsr().indptr).max())
            check_elementwise(outp32.cpu().numpy(), (P @ e32.T).T, abs_terms(P, e32), fp16_coef(nt),
                              "prolong mixed k=%d nrhs=%d" % (k, nr))
    for level in (1, 2):
        n = gh.ndof(level)
        v = gaussian_vectors(nrhs, n, 50 + level)
        A = oh.ops[level]
        for dag, ref in ((False, A), (True, A.conj().T)):
            out = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
            K.kdmg_coarse_apply(gh, level, dev(v), out, nrhs, dagger=dag)
            torch.cuda.synchronize()
            assert relerr(out.cpu().numpy(), (ref @ v.T).T) < 1e-12
            out32 = torch.empty((nrhs, n), dtype=torch.complex64, device="cuda")
            K.kdmg_coarse_apply(gh, level, dev(v, torch.complex64), out32, nrhs, dagger=dag,
                                prec=K.KDMG_MIXED)
            torch.cuda.synchronize()
            v32 = rounded(v)
            nt = int(np.diff(ref.tocsr().indptr).max())
            check_elementwise(out32.cpu().numpy(), (ref @ v32.T).T, abs_terms(ref, v32), fp32_coef(nt),
                              "coarse apply mixed level %d dag %d" % (level, dag))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_level_solve_c1(K, prec):
    """16^2, beta=3, m=0.1, 2 levels (4x4 KD-block aggregates, n_vec 8): the
    small workload; dense LU is the exact answer."""
    dims, beta, m = (16, 16), 3.0, 0.1
    U = field(dims, beta, seed=101, sweeps=200)
    levels = [((4, 4), 8)]
    oh, psi0 = oracle_setup(dims, U, m, levels, 7)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), psi0)
    b = gaussian_vectors(1, lat.volume, 55)
    x = torch.empty((1, lat.volume), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, 1, 1e-10, prec=p)
    xg = x.cpu().numpy()[0]
    xd = dense_solve(OLattice(dims), U, m, b[0])
    assert info[0]["converged"] and info[0]["true_rel_resid"] <= 1e-10
    D = dirac_matrix(OLattice(dims), U, m)
    assert np.linalg.norm(b[0] - D @ xg) / np.linalg.norm(b[0]) <= 1e-10
    assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) < 1e-8
    xo, oinfo = OSolver(oh).solve(b[0], 1e-10)
    if prec == "fp64":
        assert abs(info[0]["outer_its"] - oinfo["outer_its"]) <= 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_three_level_multi_rhs_solve(K, prec):
    dims, beta, m = (32, 32), 6.0, 0.02
    U = field(dims, beta, seed=102, sweeps=100)
    levels = [((2, 2), 8), ((2, 2), 8)]
    oh, psi0 = oracle_setup(dims, U, m, levels, 8)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), psi0)
    nrhs = 4
    b = gaussian_vectors(nrhs, lat.volume, 56)
    x = torch.empty((nrhs, lat.volume), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, nrhs, 1e-10, prec=p)
    D = dirac_matrix(OLattice(dims), U, m)
    xs = x.cpu().numpy()
    for r in range(nrhs):
        assert info[r]["converged"]
        assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
        xd = dense_solve(OLattice(dims), U, m, b[r])
        assert np.linalg.norm(xs[r] - xd) / np.linalg.norm(xd) < 1e-8
    # each rhs alone gives the same answer as in the batch
    x1 = torch.empty((1, lat.volume), dtype=torch.complex128, device="cuda")
    info1, _ = K.kdmg_solve(gh, dev(b[2:3]), x1, 1, 1e-10, prec=p)
    assert info1[0]["outer_its"] == info[2]["outer_its"]
    assert np.linalg.norm(x1.cpu().numpy()[0] - xs[2]) / np.linalg.norm(xs[2]) < 1e-12


def test_outer_stall_rule(K):
    """The opt-in stall rule of the outer solve (a serving policy): with a
    working hierarchy that halves the residual every iteration it never fires
    and the result is bit-identical to the solve without it; with a crippled
    preconditioner (one intermediate and one coarsest iteration, no
    smoothing) and a 2-iteration window it stops every rhs after 2 outer
    iterations with KDMG_ENOCONV, the returned iterate no worse than x = 0."""
    dims, beta, m = (32, 32), 6.0, 0.02
    U = field(dims, beta, seed=102, sweeps=100)
    levels = [((2, 2), 8), ((2, 2), 8)]
    _, psi0 = oracle_setup(dims, U, m, levels, 8)
    lat = K.Lattice(dims, U)
    b = gaussian_vectors(3, lat.volume, 57)
    D = dirac_matrix(OLattice(dims), U, m)
    xs = []
    for stall in (0, 4):
        gh = K.Hierarchy(lat, m, K.make_params(levels, outer_stall=stall), psi0)
        x = torch.empty((3, lat.volume), dtype=torch.complex128, device="cuda")
        info, _ = K.kdmg_solve(gh, dev(b), x, 3, 1e-10, prec=K.KDMG_FP64)
        assert all(i["converged"] for i in info)
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
    weak = K.make_params(levels, outer_stall=2, inter_maxit=1, coarse_maxit=1, mr_its=0, outer_maxit=50)
    gh = K.Hierarchy(lat, 0.001, weak, psi0)
    x = torch.empty((3, lat.volume), dtype=torch.complex128, device="cuda")
    info, st = K.kdmg_solve(gh, dev(b), x, 3, 1e-10, prec=K.KDMG_FP64, raise_on_noconv=False)
    assert st == K.KDMG_ENOCONV
    D0 = dirac_matrix(OLattice(dims), U, 0.001)
    xw = x.cpu().numpy()
    for r in range(3):
        assert not info[r]["converged"] and info[r]["outer_its"] == 2
        assert np.linalg.norm(b[r] - D0 @ xw[r]) <= np.linalg.norm(b[r])


def test_free_field_solve_matches_fft(K):
    from oracle.exact import free_fft_solve
    dims, m = (32, 32), 0.01
    U = unit_gauge(dims)
    levels = [((4, 4), 8)]
    oh, psi0 = oracle_setup(dims, U, m, levels, 9)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), psi0)
    b = gaussian_vectors(1, lat.volume, 57)
    x = torch.empty((1, lat.volume), dtype=torch.complex128, device="cuda")
    info, _ = K.kdmg_solve(gh, dev(b), x, 1, 1e-10)
    xf = free_fft_solve(OLattice(dims), m, b[0])
    assert np.linalg.norm(x.cpu().numpy()[0] - xf) / np.linalg.norm(xf) < 1e-8


def test_errors_are_reported(K):
    dims = (16, 16)
    U = field(dims, 3.0)
    with pytest.raises(K.KdmgError) as e:
        K.Lattice((10, 16), unit_gauge((10, 16)))
    assert e.value.status == K.KDMG_EINVAL
    lat = K.Lattice(dims, U)
    bad = K.make_params([((3, 3), 8)])  # 3 does not divide the 8x8 block lattice
    with pytest.raises(K.KdmgError) as e:
        K.Hierarchy(lat, 0.1, bad, [gaussian_vectors(8, 256, 1)])
    assert e.value.status == K.KDMG_EINVAL
    with pytest.raises(K.KdmgError) as e:
        K.Hierarchy(lat, 0.1, K.make_params([((4, 4), 8)], outer_stall=-1), [gaussian_vectors(8, 256, 1)])
    for bad in (-1, 65):
        with pytest.raises(K.KdmgError):
            K.Hierarchy(lat, 0.1, K.make_params([((4, 4), 8)], coarse_tail=bad), [gaussian_vectors(8, 256, 1)])
    assert e.value.status == K.KDMG_EINVAL
    # iteration cap forced from the host: ENOCONV with the best iterate returned
    levels = [((4, 4), 8)]
    p = K.make_params(levels, outer_maxit=1)
    h = K.Hierarchy(lat, 0.1, p, [gaussian_vectors(8, 256, 2, tag=1)])
    b = gaussian_vectors(1, 256, 3)
    x = torch.empty((1, 256), dtype=torch.complex128, device="cuda")
    info, st = K.kdmg_solve(h, dev(b), x, 1, 1e-10, raise_on_noconv=False)
    assert st == K.KDMG_ENOCONV and not info[0]["converged"]
    assert info[0]["true_rel_resid"] < 1.0


@pytest.mark.parametrize("nv", [8, 12])
@pytest.mark.parametrize("nrhs", [1, 5, 16, 33])
def test_coarse_apply_all_shapes(K, nv, nrhs):
    """Coarse stencil apply and adjoint for every launch shape (SIMT tiles for
    < 16 rhs, MFMA 16x16x4 tiles for >= 16 rhs, padded when 2 n_vec is not a
    multiple of 16), FP64 and FP32, against the oracle's sparse operator."""
    dims, beta, m = (32, 32), 6.0, 0.02
    levels = [((4, 4), nv), ((2, 2), nv)]
    U = field(dims, beta)
    oh, _ = oracle_setup(dims, U, m, levels, 24)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), oh.nullvecs, relaxed=True)
    for level in (1, 2):
        n = gh.ndof(level)
        v = gaussian_vectors(nrhs, n, 60 + level + nrhs)
        A = oh.ops[level]
        for dag, ref in ((False, A), (True, A.conj().T)):
            r = (ref @ v.T).T
            out = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
            K.kdmg_coarse_apply(gh, level, dev(v), out, nrhs, dagger=dag)
            torch.cuda.synchronize()
            assert relerr(out.cpu().numpy(), r) < 1e-12
            out32 = torch.empty((nrhs, n), dtype=torch.complex64, device="cuda")
            K.kdmg_coarse_apply(gh, level, dev(v, torch.complex64), out32, nrhs, dagger=dag,
                                prec=K.KDMG_MIXED)
            torch.cuda.synchronize()
            v32 = rounded(v)
            nt = int(np.diff(ref.tocsr().indptr).max())
            check_elementwise(out32.cpu().numpy(), (ref @ v32.T).T, abs_terms(ref, v32), fp32_coef(nt),
                              "coarse apply shapes level %d dag %d" % (level, dag))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_solve_mfma_path(K, prec):
    """20 rhs (MFMA stencil tiles and fused CGNE) on 32^2, three levels with
    n_vec 8 then 12: every rhs reaches 1e-10 and matches dense LU to 1e-8.
    The coarsest CGNE calls continue as a 16-rhs tail problem once 16 or
    fewer rhs remain active (the default coarse_tail); with the tail off the
    same solve gives outer iteration counts within one and agrees to 1e-9 (the
    tail runs its own launch shape, so rounding may differ)."""
    dims, beta, m = (32, 32), 6.0, 0.02
    U = field(dims, beta, seed=103, sweeps=100)
    levels = [((2, 2), 8), ((2, 2), 12)]
    oh, psi0 = oracle_setup(dims, U, m, levels, 9)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), psi0)
    nrhs = 20
    b = gaussian_vectors(nrhs, lat.volume, 58)
    x = torch.empty((nrhs, lat.volume), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, nrhs, 1e-10, prec=p)
    D = dirac_matrix(OLattice(dims), U, m).toarray()
    xd = np.linalg.solve(D, b.T).T
    xs = x.cpu().numpy()
    for r in range(nrhs):
        assert info[r]["converged"]
        assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
        assert np.linalg.norm(xs[r] - xd[r]) / np.linalg.norm(xd[r]) < 1e-8
    assert gh.counters()["tail_entries"] > 0
    g0 = K.Hierarchy(lat, m, gpu_params(K, levels, coarse_tail=0), psi0)
    x0 = torch.empty_like(x)
    info0, _ = K.kdmg_solve(g0, dev(b), x0, nrhs, 1e-10, prec=p)
    assert g0.counters()["tail_entries"] == 0
    x0 = x0.cpu().numpy()
    for r in range(nrhs):
        assert info0[r]["converged"]
        assert abs(info0[r]["outer_its"] - info[r]["outer_its"]) <= 1
        assert np.linalg.norm(x0[r] - xs[r]) / np.linalg.norm(xs[r]) < 1e-9


def test_hierarchy_at_mass_and_rebind(K):
    """kdmg_hierarchy_at_mass / kdmg_hierarchy_set_mass: coarse operators
    Galerkin-built at a new mass from the same null vectors equal the oracle's
    (built from those vectors at that mass) to rounding; moving back to the
    first mass reproduces the first operators bit for bit; moving onto another
    configuration of the same shape equals that configuration's oracle; the
    moved hierarchy solves to 1e-10 and matches dense LU."""
    dims, beta, m0, m1 = (32, 32), 6.0, 0.02, 0.15
    levels = [((2, 2), 8), ((2, 2), 8)]
    olevels = MGParams(levels=[LevelParams(a, nv) for a, nv in levels])
    olat = OLattice(dims)
    U = field(dims, beta)
    oh0, _ = oracle_setup(dims, U, m0, levels, 21)
    lat = K.Lattice(dims, U)
    base = K.Hierarchy(lat, m0, gpu_params(K, levels), oh0.nullvecs, relaxed=True)
    oh1 = OHierarchy(olat, U, m1, olevels, [("relaxed", v) for v in oh0.nullvecs])
    h = base.at_mass(m1)
    for k in (1, 2):
        dims_c, _ = h.level_info(k)
        assert relerr(assemble(h.coarse_op(k), dims_c), oh1.ops[k].toarray()) < 1e-11
    h.set_mass(m0)
    for k in (1, 2):
        assert np.array_equal(h.coarse_op(k), base.coarse_op(k))
    U2 = field(dims, beta, seed=8)
    oh2, _ = oracle_setup(dims, U2, m0, levels, 22)
    lat2 = K.Lattice(dims, U2)
    base2 = K.Hierarchy(lat2, m0, gpu_params(K, levels), oh2.nullvecs, relaxed=True)
    h.set_mass(m1, base=base2)
    oh2b = OHierarchy(olat, U2, m1, olevels, [("relaxed", v) for v in oh2.nullvecs])
    for k in (1, 2):
        dims_c, _ = h.level_info(k)
        assert relerr(assemble(h.coarse_op(k), dims_c), oh2b.ops[k].toarray()) < 1e-11
    b = gaussian_vectors(2, olat.volume, 5, tag=0)
    x = torch.empty((2, olat.volume), dtype=torch.complex128, device="cuda")
    for prec in (K.KDMG_FP64, K.KDMG_MIXED):
        info, _ = K.kdmg_solve(h, dev(b), x, 2, 1e-10, prec=prec)
        xs = x.cpu().numpy()
        D = dirac_matrix(olat, U2, m1)
        for r in range(2):
            assert info[r]["converged"]
            assert np.linalg.norm(b[r] - D @ xs[r]) / np.linalg.norm(b[r]) <= 1e-10
            xd = dense_solve(olat, U2, m1, b[r])
            assert np.linalg.norm(xs[r] - xd) / np.linalg.norm(xd) < 1e-8
    other = K.Hierarchy(K.Lattice((16, 32), field((16, 32), beta)), m0, gpu_params(K, levels),
                        oracle_setup((16, 32), field((16, 32), beta), m0, levels, 23)[0].nullvecs,
                        relaxed=True)
    with pytest.raises(K.KdmgError) as e:
        h.set_mass(m0, base=other)
    assert e.value.status == K.KDMG_EINVAL


def test_cgne_graph_replay_matches_eager(K):
    """The coarsest CGNE replays captured hipGraph chunks (the default); with
    eager launches and host work between every replay, the same solve gives
    bit-identical results, solve after solve (several hundred replays)."""
    dims, beta, m = (64, 64), 6.0, 0.01
    levels = [((4, 4), 8), ((2, 2), 12)]
    U = field(dims, beta)
    oh, _ = oracle_setup(dims, U, m, levels, 31)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), oh.nullvecs, relaxed=True)
    nrhs = 20
    b = dev(gaussian_vectors(nrhs, dims[0] * dims[1], 8, tag=0))
    outs = {}
    for graphs in (False, True, True, False, True):
        gh.graphs(graphs)
        x = torch.zeros_like(b)
        info, _ = K.kdmg_solve(gh, b, x, nrhs, 1e-10, prec=K.KDMG_MIXED)
        assert all(i["converged"] for i in info)
        outs.setdefault(graphs, []).append(x.cpu().numpy())
    assert gh.graphs() > 0  # chunks were really replayed
    ref = outs[False][0]
    for arrs in outs.values():
        for a in arrs:
            assert np.array_equal(a, ref)


@pytest.mark.parametrize("nv,nrhs", [(12, 32), (8, 20), (12, 5)])
def test_every_tuner_candidate(K, nv, nrhs):
    """Every launch shape the autotuner may choose (MFMA tiles with and
    without staged blocks and with 1-4 way k-splits, SIMT tiles) gives the
    coarse stencil and its adjoint, FP64 and FP32, to the oracle's bar."""
    dims, beta, m = (32, 32), 6.0, 0.02
    levels = [((4, 4), nv), ((2, 2), nv)]
    U = field(dims, beta)
    oh, _ = oracle_setup(dims, U, m, levels, 25)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, gpu_params(K, levels), oh.nullvecs, relaxed=True)
    for level in (1, 2):
        n = gh.ndof(level)
        v = gaussian_vectors(nrhs, n, 70 + level + nrhs)
        A = oh.ops[level]
        for dag, ref in ((False, A), (True, A.conj().T)):
            r = (ref @ v.T).T
            v32 = rounded(v)
            r32 = (ref @ v32.T).T
            t32 = abs_terms(ref, v32)
            c32 = fp32_coef(int(np.diff(ref.tocsr().indptr).max()))
            for prec, dt in ((K.KDMG_FP64, torch.complex128), (K.KDMG_MIXED, torch.complex64)):
                out = torch.empty((64, nrhs, n), dtype=dt, device="cuda")
                nc = K.kdmg_coarse_apply_candidates(gh, level, dev(v, dt), out, nrhs, dagger=dag, prec=prec)
                assert 1 <= nc <= 64
                got = out[:nc].cpu().numpy()
                for c in range(nc):
                    if prec == K.KDMG_FP64:
                        assert relerr(got[c], r) < 1e-12, c
                    else:
                        check_elementwise(got[c], r32, t32, c32, "candidate %d" % c)
