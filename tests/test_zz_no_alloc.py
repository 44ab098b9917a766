"""kdmg_apply_schur_noalloc (the entry point for callers that cannot
allocate) against kdmg_apply_schur through the C ABI: two calls in a row,
the second on a smaller input, each bit-identical to the allocating entry
point (same kernels, same launch shapes) and within 1e-12 of the oracle's
Schur operator; a request above the fixed work space is refused before any
device work."""
import numpy as np
import pytest

from oracle.staggered import Lattice as OLattice
from oracle.kd import KDOperator
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


def _case(K, dims, beta, m, nrhs, seed):
    U, _ = u1_heatbath(dims, beta, 30, seed)
    lat = K.Lattice(dims, U)
    nh = lat.volume // 2
    v = gaussian_vectors(nrhs, nh, seed, tag=4)
    vin = torch.from_numpy(v).to("cuda")
    out_a = torch.full_like(vin, complex(np.nan, np.nan))
    out_n = torch.full_like(vin, complex(np.nan, np.nan))
    K.kdmg_apply_schur(lat, m, vin, out_a, nrhs)
    K.kdmg_apply_schur_noalloc(lat, m, vin, out_n, nrhs)
    torch.cuda.synchronize()
    assert torch.equal(out_a, out_n)
    kd = KDOperator(OLattice(dims), U, m)
    ref = (kd.S @ v.T).T
    got = out_n.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    return lat


def test_noalloc_schur_matches_allocating_entry_point(K):
    lat = _case(K, (64, 64), 6.0, 0.05, 7, 31)
    _case(K, (32, 32), 3.0, 0.2, 2, 32)   # second call, smaller input
    # more rhs than the fixed work space holds: refused, nothing launched
    nmax = (32 << 20) // (6 * (lat.volume // 2) * 16)
    big = torch.zeros((nmax + 1, lat.volume // 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(K.KdmgError) as e:
        K.kdmg_apply_schur_noalloc(lat, 0.05, big, torch.empty_like(big), nmax + 1)
    assert e.value.status == K.KDMG_EINVAL
