"""The solve service (kdmg_server_*): requests over resident configurations,
admitted as workers and memory free up, running concurrently on separate
streams.  Checked here:
  * every served result solves D x = b to 1e-10 (residual recomputed with the
    oracle's D in FP64 on the CPU);
  * each result is the same alone (one worker, one request at a time) and in
    the mix (three workers, all requests queued at once): relative difference
    <= 1e-12 (the path is deterministic, so in practice identical);
  * served results equal a direct kdmg_hierarchy_at_mass + kdmg_solve;
  * admission: with a budget for one request at a time, no two run together
    and the reserved bytes never exceed the budget; a request larger than the
    budget is refused with KDMG_ENOMEM.
"""
import numpy as np
import pytest

from oracle.staggered import Lattice as OLattice, dirac_matrix
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


SERVED = [((16, 16), 3.0, 11, [((4, 4), 8)]),
           ((32, 32), 6.0, 12, [((2, 2), 8), ((2, 2), 8)]),
           ((32, 32), 6.0, 13, [((2, 2), 8), ((2, 2), 8)])]
M_SETUP = 0.02


@pytest.fixture(scope="module")
def served(K):
    out = []
    for dims, beta, seed, levels in SERVED:
        U, _ = u1_heatbath(dims, beta, 30, seed)
        lat = K.Lattice(dims, U)
        psi0 = []
        n = dims[0] * dims[1]
        nsites = n // 4
        for k, (agg, nv) in enumerate(levels):
            psi0.append(gaussian_vectors(nv, n, seed, tag=1 + k))
            nsites //= int(np.prod(agg))
            n = nsites * 2 * nv
        h = K.Hierarchy(lat, M_SETUP, K.make_params(levels), psi0)
        out.append((dims, U, lat, h))
    return out


def requests(served, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        c = int(rng.integers(len(served)))
        m = float(np.exp(rng.uniform(np.log(0.01), np.log(0.1))))
        V = int(np.prod(served[c][0]))
        b = gaussian_vectors(1, V, 900 + seed, tag=i)
        reqs.append((c, m, b))
    return reqs


def serve(K, served, reqs, slots, budget, all_at_once):
    srv = K.Server(slots, budget)
    ids = [srv.add_config(h) for (_, _, _, h) in served]
    xs, infos, stats = [None] * len(reqs), [None] * len(reqs), None
    try:
        tickets = []
        bufs = []
        for i, (c, m, b) in enumerate(reqs):
            bd = torch.from_numpy(b).to("cuda")
            xd = torch.zeros_like(bd)
            bufs.append((bd, xd))
            t = srv.submit(ids[c], m, bd, xd, 1, 1e-10, K.KDMG_MIXED)
            if all_at_once:
                tickets.append(t)
            else:
                st, info, _ = srv.poll(t, wait=True)
                assert st == K.KDMG_OK, srv.last_error
                xs[i], infos[i] = xd.cpu().numpy()[0], info[0]
        for i, t in enumerate(tickets):
            st, info, _ = srv.poll(t, wait=True)
            assert st == K.KDMG_OK, srv.last_error
            xs[i], infos[i] = bufs[i][1].cpu().numpy()[0], info[0]
        stats = srv.stats()
    finally:
        srv.close()
    return xs, infos, stats


def test_served_alone_equals_mix(K, served):
    reqs = requests(served, 12, 1)
    budget = 8 << 30
    x_alone, _, st_alone = serve(K, served, reqs, 1, budget, all_at_once=False)
    x_mix, info_mix, st_mix = serve(K, served, reqs, 3, budget, all_at_once=True)
    assert st_alone["peak_running"] == 1
    assert st_mix["peak_running"] >= 2
    assert st_mix["completed"] == len(reqs)
    exact = 0
    for (c, m, b), xa, xm, inf in zip(reqs, x_alone, x_mix, info_mix):
        dims, U = served[c][0], served[c][1]
        D = dirac_matrix(OLattice(dims), U, m)
        assert inf["converged"]
        assert np.linalg.norm(b[0] - D @ xm) / np.linalg.norm(b[0]) <= 1e-10
        assert np.linalg.norm(xm - xa) / np.linalg.norm(xa) <= 1e-12
        exact += int(np.array_equal(xm, xa))
    print("served results identical alone and in the mix: %d of %d" % (exact, len(reqs)))


def test_served_equals_direct_solve(K, served):
    reqs = requests(served, 4, 2)
    x_srv, _, _ = serve(K, served, reqs, 2, 8 << 30, all_at_once=True)
    for (c, m, b), xs in zip(reqs, x_srv):
        h = served[c][3].at_mass(m)
        bd = torch.from_numpy(b).to("cuda")
        xd = torch.zeros_like(bd)
        info, _ = K.kdmg_solve(h, bd, xd, 1, 1e-10, prec=K.KDMG_MIXED)
        x = xd.cpu().numpy()[0]
        assert np.linalg.norm(xs - x) / np.linalg.norm(x) <= 1e-12


def test_admission_by_footprint(K, served):
    reqs = [r for r in requests(served, 10, 3) if r[0] != 0][:5]
    srv = K.Server(3, 1 << 40)
    cid = srv.add_config(served[1][3])
    one = srv.request_bytes(cid, 1, K.KDMG_MIXED)
    srv.close()
    budget = int(one * 1.5)
    _, infos, st = serve(K, served, reqs, 3, budget, all_at_once=True)
    assert all(i["converged"] for i in infos)
    assert st["peak_running"] == 1
    assert st["peak_allocated"] <= budget
    small = K.Server(2, one // 2)
    try:
        c = small.add_config(served[1][3])
        b = torch.zeros((1, 32 * 32), dtype=torch.complex128, device="cuda")
        x = torch.zeros_like(b)
        with pytest.raises(K.KdmgError) as e:
            small.submit(c, 0.05, b, x)
        assert e.value.status == K.KDMG_ENOMEM
    finally:
        small.close()


def test_served_exact_coarsest_first_requests(K):
    """Configurations with the exact coarsest solve, every request queued at
    once on fresh configurations, so the first requests of each tune launch
    shapes while other workers solve: every request succeeds (served solves
    run without graph capture), reaches 1e-10, and equals a direct solve."""
    cfgs = []
    for dims, beta, seed, levels in SERVED:
        U, _ = u1_heatbath(dims, beta, 30, seed + 100)
        lat = K.Lattice(dims, U)
        psi0 = []
        n = dims[0] * dims[1]
        nsites = n // 4
        for k, (agg, nv) in enumerate(levels):
            psi0.append(gaussian_vectors(nv, n, seed, tag=1 + k))
            nsites //= int(np.prod(agg))
            n = nsites * 2 * nv
        h = K.Hierarchy(lat, M_SETUP, K.make_params(levels, coarse_solver=1), psi0)
        cfgs.append((dims, U, lat, h))
    reqs = requests(cfgs, 12, 4)
    xs, infos, st = serve(K, cfgs, reqs, 4, 8 << 30, all_at_once=True)
    assert st["completed"] == len(reqs)
    for (c, m, b), x, inf in zip(reqs, xs, infos):
        dims, U = cfgs[c][0], cfgs[c][1]
        D = dirac_matrix(OLattice(dims), U, m)
        assert inf["converged"]
        assert np.linalg.norm(b[0] - D @ x) / np.linalg.norm(b[0]) <= 1e-10
        h = cfgs[c][3].at_mass(m)
        bd = torch.from_numpy(b).to("cuda")
        xd = torch.zeros_like(bd)
        K.kdmg_solve(h, bd, xd, 1, 1e-10, prec=K.KDMG_MIXED)
        xr = xd.cpu().numpy()[0]
        assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-12
