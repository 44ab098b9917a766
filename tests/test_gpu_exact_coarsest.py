"""GPU parity of the exact coarsest solve (kdmg_mg_params.coarse_solver = 1,
an option beside Table 1's CGNE(0.2)): the explicit inverse built on the GPU
(FP64 Gauss-Jordan on A A^dag, then A^dag N^-1) against the oracle's dense LU
solve of its own coarsest operator, from identical relaxed null vectors, and
the full KD-MG solve with it against dense LU and the oracle's K-cycle with
the same option.

Tolerance of the coarsest solve: the two coarsest operators agree to about
1e-12 relative (same vectors, different summation order), the GPU inverse
carries kappa(A)^2 * 1e-16 from the normal equations, so the solutions agree
to kappa(A) * 1e-12 + kappa(A)^2 * 1e-16; at these masses kappa(A) < 100 and
the bar is 1e-9."""
import numpy as np
import pytest
import scipy.linalg

from oracle.staggered import Lattice as OLattice, dirac_matrix
from oracle.mg import MGParams, LevelParams, Hierarchy as OHierarchy, Solver as OSolver
from oracle.exact import dense_solve
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.complex128)


def setup(dims, beta, m, levels, seed, sweeps=100):
    U, _ = u1_heatbath(dims, beta, sweeps, seed)
    olat = OLattice(dims)
    psi0 = []
    n, ncs = olat.ndof, None
    for k, (agg, nv) in enumerate(levels):
        psi0.append(gaussian_vectors(nv, n, seed, tag=1 + k))
        ncs = olat.volume // int(np.prod([2 * a for a in agg])) if k == 0 else ncs // int(np.prod(agg))
        n = ncs * 2 * nv
    oh = OHierarchy(olat, U, m, MGParams(levels=[LevelParams(a, nv) for a, nv in levels], coarse_exact=True),
                    psi0)
    return U, oh, psi0


# (dims, beta, m, levels, nrhs): coarsest sizes 64, 336 (not a multiple of
# 32: ragged row tiles and k-splits) and 256; rhs counts on both MFMA tile
# widths, with ragged tails
CASES = [((16, 16), 3.0, 0.1, [((4, 4), 8)], 1),
         ((24, 16), 6.0, 0.05, [((2, 2), 7)], 20),
         ((32, 32), 6.0, 0.02, [((2, 2), 8), ((2, 2), 8)], 33)]


@pytest.mark.parametrize("dims,beta,m,levels,nrhs", CASES)
def test_coarsest_inverse_matches_oracle_lu(K, dims, beta, m, levels, nrhs):
    U, oh, _ = setup(dims, beta, m, levels, 21)
    lat = K.Lattice(dims, U)
    relaxed = [v for v in oh.nullvecs]
    gh = K.Hierarchy(lat, m, K.make_params(levels, coarse_solver=1), relaxed, relaxed=True)
    top = gh.nlevels - 1
    A = oh.ops[top].toarray()
    n = A.shape[0]
    assert gh.ndof(top) == n
    r = gaussian_vectors(nrhs, n, 5, tag=3)
    out = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
    K.kdmg_coarsest_solve(gh, dev(r), out, nrhs)
    xg = out.cpu().numpy()
    lu = scipy.linalg.lu_factor(A)
    for q in range(nrhs):
        xo = scipy.linalg.lu_solve(lu, r[q])
        assert np.linalg.norm(xg[q] - xo) / np.linalg.norm(xo) <= 1e-9, q
        assert np.linalg.norm(A @ xg[q] - r[q]) / np.linalg.norm(r[q]) <= 1e-10, q


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_with_exact_coarsest(K, prec):
    """Three-level solve with the exact coarsest option: every rhs reaches
    1e-10 and the dense-LU solution to 1e-8; in FP64 the outer count is
    within one of the oracle's K-cycle with its dense coarsest LU."""
    dims, beta, m = (32, 32), 6.0, 0.02
    levels = [((2, 2), 8), ((2, 2), 8)]
    U, oh, psi0 = setup(dims, beta, m, levels, 8)
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m, K.make_params(levels, coarse_solver=1), psi0)
    nrhs = 5
    b = gaussian_vectors(nrhs, lat.volume, 56)
    x = torch.empty((nrhs, lat.volume), dtype=torch.complex128, device="cuda")
    p = K.KDMG_FP64 if prec == "fp64" else K.KDMG_MIXED
    info, _ = K.kdmg_solve(gh, dev(b), x, nrhs, 1e-10, prec=p)
    D = dirac_matrix(OLattice(dims), U, m)
    xs = x.cpu().numpy()
    for q in range(nrhs):
        assert info[q]["converged"] and info[q]["level_avg_its"][1] == 1.0
        assert np.linalg.norm(b[q] - D @ xs[q]) / np.linalg.norm(b[q]) <= 1e-10
        xd = dense_solve(OLattice(dims), U, m, b[q])
        assert np.linalg.norm(xs[q] - xd) / np.linalg.norm(xd) <= 1e-8
    if prec == "fp64":
        _, oinfo = OSolver(oh).solve(b[0], 1e-10)
        assert abs(info[0]["outer_its"] - oinfo["outer_its"]) <= 1, (info[0], oinfo)


def test_exact_coarsest_follows_mass_change(K):
    """kdmg_hierarchy_set_mass rebuilds the inverse at the new mass."""
    dims, beta, m0, m1 = (24, 16), 6.0, 0.05, 0.2
    levels = [((2, 2), 7)]
    U, oh0, _ = setup(dims, beta, m0, levels, 21)
    relaxed = [v for v in oh0.nullvecs]
    oh1 = OHierarchy(OLattice(dims), U, m1, MGParams(levels=[LevelParams(a, nv) for a, nv in levels],
                                                     coarse_exact=True), [("relaxed", v) for v in relaxed])
    lat = K.Lattice(dims, U)
    gh = K.Hierarchy(lat, m0, K.make_params(levels, coarse_solver=1), relaxed, relaxed=True)
    gh.set_mass(m1)
    A1 = oh1.ops[1].toarray()
    r = gaussian_vectors(3, A1.shape[0], 6, tag=3)
    out = torch.empty((3, A1.shape[0]), dtype=torch.complex128, device="cuda")
    K.kdmg_coarsest_solve(gh, dev(r), out, 3)
    xg = out.cpu().numpy()
    for q in range(3):
        xo = np.linalg.solve(A1, r[q])
        assert np.linalg.norm(xg[q] - xo) / np.linalg.norm(xo) <= 1e-9


def test_kcycle_graphs_match_eager(K):
    """With the exact coarsest solve, the intermediate level's K-cycle has no
    host decision below it, and its two halves around the coarsest product
    replay as captured hipGraphs: the replayed solve equals the plainly
    launched one bit for bit, on repeated solves with other work between
    them, and after a rebind to another configuration (graphs recaptured).
    In that mode the intermediate GCR also defers its host poll of the
    convergence flags to the iteration count of its previous call (iterations
    past convergence are device no-ops): the per-rhs iteration statistics
    agree too."""
    dims, beta, m = (32, 32), 6.0, 0.02
    levels = [((2, 2), 8), ((2, 2), 8)]
    U, oh, psi0 = setup(dims, beta, m, levels, 8)
    U2, _, psi2 = setup(dims, beta, m, levels, 9)
    lat, lat2 = K.Lattice(dims, U), K.Lattice(dims, U2)
    nrhs = 5
    b = dev(gaussian_vectors(nrhs, lat.volume, 57))
    res = {}
    for graphs in (True, False):
        gh = K.Hierarchy(lat, m, K.make_params(levels, coarse_solver=1), psi0)
        gh.graphs(graphs)
        xs, stats = [], []
        for rep in range(3):
            x = torch.empty_like(b)
            info, _ = K.kdmg_solve(gh, b, x, nrhs, 1e-10, prec=K.KDMG_MIXED)
            assert all(i["converged"] for i in info)
            xs.append(x.clone())
            stats.append([(i["outer_its"], tuple(i["level_avg_its"])) for i in info])
            torch.cuda.synchronize()
            _ = (b * 2.0).sum()  # unrelated work between replays
        replays = gh.counters()["graph_replays"]
        assert (replays > 0) == graphs
        # rebind to another configuration and back: graphs recaptured
        other = K.Hierarchy(lat2, m, K.make_params(levels, coarse_solver=1), psi2)
        gh.set_mass(m, base=other)
        x2 = torch.empty_like(b)
        info2, _ = K.kdmg_solve(gh, b, x2, nrhs, 1e-10, prec=K.KDMG_MIXED)
        assert all(i["converged"] for i in info2)
        res[graphs] = (xs, x2, stats)
    for rep in range(3):
        assert torch.equal(res[True][0][rep], res[False][0][0])
        assert res[True][2][rep] == res[False][2][0]
    assert torch.equal(res[True][1], res[False][1])
