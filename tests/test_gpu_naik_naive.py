"""GPU parity of the Naik-improved operator and its KD multigrid (Sec. 2.1,
eq. "freehisq"), and of Galerkin multigrid on D itself, the negative control
of Sec. 3.2 (kdmg_mg_params.fine_op = 1), against the FP64 oracle on the same
seeded inputs.

Bars: FP64 operators <= 1e-12 relative max-norm; the FP16-link form element
by element within 2^-11 (plus FP32 accumulation) times the sum of the
absolute terms; P and the coarse operators from the oracle's relaxed vectors
<= 1e-11; solves: true residual <= 1e-10 with the oracle's operator, the
dense-LU solution to 1e-8, FP64 outer iteration counts within one of the
oracle's K-cycle."""
import numpy as np
import pytest

from oracle.staggered import Lattice as OLattice, dirac_matrix, dirac_matrix_naik
from oracle.kd import KDOperator
from oracle.mg import MGParams, LevelParams, Hierarchy as OHierarchy, Solver as OSolver
from mixed_bounds import fp16_coef, abs_terms, rounded, check_elementwise
from synth import u1_heatbath, gaussian_vectors

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


def field(dims, beta=6.0, seed=31, sweeps=60):
    U, _ = u1_heatbath(dims, beta, sweeps, seed)
    return U


def naik_lattice(K, dims, U):
    lat = K.Lattice(dims, U)
    lat.set_naik(True)
    return lat


@pytest.mark.parametrize("dims,bc", [((16, 16), None), ((24, 16), (-1, -1))])
def test_naik_apply_D(K, dims, bc):
    U = field(dims)
    olat = OLattice(dims, bc=bc)
    lat = K.Lattice(dims, U, bc=bc)
    lat.set_naik(True)
    m = 0.07
    D = dirac_matrix_naik(olat, U, m)
    nr = 3
    v = gaussian_vectors(nr, lat.volume, 8)
    out = torch.empty((nr, lat.volume), dtype=torch.complex128, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v), out, nr)
    assert relerr(out.cpu().numpy(), (D @ v.T).T) < 1e-12
    out32 = torch.empty((nr, lat.volume), dtype=torch.complex64, device="cuda")
    K.kdmg_apply_D(lat, m, dev(v, torch.complex64), out32, nr, prec=K.KDMG_MIXED)
    v32 = rounded(v)
    check_elementwise(out32.cpu().numpy(), (D @ v32.T).T, abs_terms(D, v32), fp16_coef(9), "Naik D mixed")
    # switching back restores eq. "staggeredD"
    lat.set_naik(False)
    K.kdmg_apply_D(lat, m, dev(v), out, nr)
    assert relerr(out.cpu().numpy(), (dirac_matrix(olat, U, m) @ v.T).T) < 1e-12


def test_naik_kd_operators(K):
    dims = (16, 16)
    U = field(dims)
    m = 0.1
    kd = KDOperator(OLattice(dims), U, m, naik=True)
    lat = naik_lattice(K, dims, U)
    nr = 2
    v = gaussian_vectors(nr, lat.volume, 9)
    for fn, ref in ((lambda i, o: K.kdmg_apply_A(lat, m, i, o, nr), kd.A),
                    (lambda i, o: K.kdmg_apply_A(lat, m, i, o, nr, dagger=True), kd.Adag),
                    (lambda i, o: K.kdmg_apply_Binv(lat, m, i, o, nr), kd.Binv)):
        out = torch.empty((nr, lat.volume), dtype=torch.complex128, device="cuda")
        fn(dev(v), out)
        torch.cuda.synchronize()
        assert relerr(out.cpu().numpy(), (ref @ v.T).T) < 1e-12
    with pytest.raises(K.KdmgError) as e:
        ve = torch.zeros((1, lat.volume // 2), dtype=torch.complex128, device="cuda")
        K.kdmg_apply_schur(lat, m, ve, torch.empty_like(ve), 1)
    assert e.value.status == K.KDMG_EUNSUPPORTED


def setup(dims, U, m, levels, seed, naik=False, fine_op="A"):
    olat = OLattice(dims)
    psi0, n, ncs = [], olat.ndof, None
    for k, (agg, nv) in enumerate(levels):
        psi0.append(gaussian_vectors(nv, n, seed, tag=1 + k))
        ncs = olat.volume // int(np.prod([2 * a for a in agg])) if k == 0 else ncs // int(np.prod(agg))
        n = ncs * 2 * nv
    oh = OHierarchy(olat, U, m, MGParams(levels=[LevelParams(a, nv) for a, nv in levels], fine_op=fine_op,
                                         outer_maxit=100), psi0, naik=naik)
    return oh, psi0


def assemble(op, dims):
    ndir, ns, nd, _ = op.shape
    M = np.zeros((ns * nd, ns * nd), dtype=np.complex128)
    L0, L1 = dims
    for Z in range(ns):
        z0, z1 = Z % L0, Z // L0
        nbrs = [Z, (z0 + 1) % L0 + L0 * z1, (z0 - 1) % L0 + L0 * z1, z0 + L0 * ((z1 + 1) % L1),
                z0 + L0 * ((z1 - 1) % L1)]
        for d in range(ndir):
            M[Z * nd:(Z + 1) * nd, nbrs[d] * nd:(nbrs[d] + 1) * nd] += op[d, Z]
    return M


@pytest.mark.parametrize("kind", ["naik", "naive"])
def test_galerkin_from_oracle_vectors(K, kind):
    """Coarse operators built on the GPU from the oracle's relaxed vectors
    equal the oracle's: A_hat = P^dag A_Naik P (with the three-link Galerkin
    term) and P^dag D P (Galerkin on D itself), levels 1 and 2."""
    dims, m = (32, 32), 0.05
    U = field(dims)
    levels = [((2, 2), 8), ((2, 2), 8)]
    naik = kind == "naik"
    oh, _ = setup(dims, U, m, levels, 12, naik=naik, fine_op="A" if naik else "D")
    lat = naik_lattice(K, dims, U) if naik else K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, K.make_params(levels, fine_op=0 if naik else 1), oh.nullvecs, relaxed=True)
    for level in (1, 2):
        dims_c, _ = gh.level_info(level)
        Ag = assemble(gh.coarse_op(level), dims_c)
        assert relerr(Ag, oh.ops[level].toarray()) < 1e-11, level


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("levels", [[((4, 4), 8)], [((2, 2), 8), ((2, 2), 8)]])
def test_naik_kd_multigrid_solve(K, prec, levels):
    dims, m = (32, 32), 0.05
    U = field(dims, seed=17)
    oh, psi0 = setup(dims, U, m, levels, 17, naik=True)
    lat = naik_lattice(K, dims, U)
    gh = K.Hierarchy(lat, m, K.make_params(levels), psi0)
    nr = 3
    b = gaussian_vectors(nr, lat.volume, 18)
    x = torch.empty((nr, lat.volume), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, nr, 1e-10, prec=p)
    D = dirac_matrix_naik(OLattice(dims), U, m)
    Dd = D.toarray()
    xs = x.cpu().numpy()
    for q in range(nr):
        assert info[q]["converged"]
        assert np.linalg.norm(b[q] - D @ xs[q]) / np.linalg.norm(b[q]) <= 1e-10
        xd = np.linalg.solve(Dd, b[q])
        assert np.linalg.norm(xs[q] - xd) / np.linalg.norm(xd) <= 1e-8
    if prec == "fp64":
        _, oinfo = OSolver(oh).solve(b[0], 1e-10)
        assert abs(info[0]["outer_its"] - oinfo["outer_its"]) <= 1, (info[0], oinfo)


def test_naive_multigrid_where_it_works(K):
    """Galerkin MG on D itself converges at a small volume and heavy mass
    (16^2, m = 0.5): the GPU path reaches the dense-LU answer, with the
    oracle's outer count."""
    dims, m = (16, 16), 0.5
    U = field(dims, seed=5)
    levels = [((2, 2), 8)]
    oh, psi0 = setup(dims, U, m, levels, 5, fine_op="D")
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, K.make_params(levels, fine_op=1), psi0)
    b = gaussian_vectors(1, lat.volume, 19)
    x = torch.empty((1, lat.volume), dtype=torch.complex128, device="cuda")
    info, _ = K.kdmg_solve(gh, dev(b), x, 1, 1e-10)
    xd = np.linalg.solve(dirac_matrix(OLattice(dims), U, m).toarray(), b[0])
    assert info[0]["converged"]
    assert np.linalg.norm(x.cpu().numpy()[0] - xd) / np.linalg.norm(xd) <= 1e-8
    _, oinfo = OSolver(oh).solve(b[0], 1e-10)
    assert oinfo["converged"] and abs(info[0]["outer_its"] - oinfo["outer_its"]) <= 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_negative_control_naive_stalls(K, prec):
    """Sec. 3.2, Fig. "residstag", on the GPU: the same three-level K-cycle
    (Table 1's parameters) on the same 32^2, beta = 6, m = 0.01 field, starts
    and rhs, coarsening D itself stalls (not converged after 100 outer
    iterations, residual above 0.1; the oracle stalls alike), while the KD
    form converges to 1e-10 in at most 25."""
    dims, m = (32, 32), 0.01
    U, _ = u1_heatbath(dims, 6.0, 200, 11)
    lat = K.Lattice(dims, U)
    levels = [((4, 4), 8), ((2, 2), 12)]
    psi0 = [gaussian_vectors(8, lat.volume, 5, tag=1), gaussian_vectors(12, (32 // 8) ** 2 * 16, 5, tag=2)]
    b = gaussian_vectors(1, lat.volume, 6)
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    res = {}
    for op in (0, 1):
        gh = K.Hierarchy(lat, m, K.make_params(levels, fine_op=op, outer_maxit=100), psi0)
        x = torch.empty((1, lat.volume), dtype=torch.complex128, device="cuda")
        info, st = K.kdmg_solve(gh, dev(b), x, 1, 1e-10, prec=p, raise_on_noconv=False)
        res[op] = info[0]
    assert res[0]["converged"] and res[0]["outer_its"] <= 25, res[0]
    assert not res[1]["converged"] and res[1]["true_rel_resid"] > 0.1, res[1]
