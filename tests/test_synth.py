"""The seeded input generators (synth/), pinned to what their definitions fix:
  * SU(3) fields: every link special unitary (U^dag U = 1, det U = 1) with
    and without APE smearing; the projection is the polar decomposition
    (idempotent on SU(3), and it recovers U from c U for c > 0); smearing
    raises the plaquette;
  * U(1) heatbath: unit-modulus links, integer topological charge, and the
    average plaquette at the exact value of 2D compact U(1) with the Wilson
    action, I1(beta) / I0(beta) (plaquettes are independent in two
    dimensions), within the statistical error of a few configurations;
  * Gaussian vectors: reproducible per (seed, tag), independent across tags,
    E|z|^2 = 2."""
import numpy as np
import pytest
from scipy.special import i0, i1

from synth import su3_smooth_random, su3_plaquette, u1_heatbath, gaussian_vectors
from synth.gauge import _proj_su3


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


@pytest.mark.parametrize("ape", [0, 2])
def test_su3_field_is_special_unitary(ape):
    U = su3_smooth_random((4, 4, 4, 4), 0.4, ape, 0.5, 17)
    assert U.shape == (4, 256, 3, 3)
    eye = np.eye(3)
    assert np.abs(_dag(U) @ U - eye).max() < 1e-12
    assert np.abs(np.linalg.det(U) - 1.0).max() < 1e-12


def test_su3_projection_is_polar():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((50, 3, 3)) + 1j * rng.standard_normal((50, 3, 3))
    W = _proj_su3(M)
    assert np.abs(_dag(W) @ W - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(W) - 1.0).max() < 1e-12
    # idempotent on SU(3), and c U -> U for c > 0
    assert np.abs(_proj_su3(W) - W).max() < 1e-12
    assert np.abs(_proj_su3(2.5 * W) - W).max() < 1e-12


def test_ape_smearing_raises_plaquette():
    dims = (4, 4, 4, 4)
    p0 = su3_plaquette(su3_smooth_random(dims, 0.8, 0, 0.5, 5), dims)
    p2 = su3_plaquette(su3_smooth_random(dims, 0.8, 2, 0.5, 5), dims)
    assert p0 < p2 <= 1.0


@pytest.mark.parametrize("beta", [3.0, 10.0])
def test_u1_heatbath_plaquette(beta):
    dims = (32, 32)
    plaq = []
    for seed in range(4):
        U, info = u1_heatbath(dims, beta, 100, 1000 + seed)
        assert np.abs(np.abs(U) - 1.0).max() < 1e-13
        q = info["topological_charge"]
        assert abs(q - round(q)) < 1e-9
        plaq.append(info["plaquette"])
    exact = i1(beta) / i0(beta)
    # 4096 independent plaquettes: the standard error is below 0.005
    assert abs(np.mean(plaq) - exact) < 0.015, (np.mean(plaq), exact)


def test_gaussian_vectors():
    a = gaussian_vectors(3, 20000, 11, tag=0)
    b = gaussian_vectors(3, 20000, 11, tag=0)
    c = gaussian_vectors(3, 20000, 11, tag=1)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    assert abs(np.mean(np.abs(a) ** 2) - 2.0) < 0.05
    assert abs(np.mean(a)) < 0.02
    # different tags are uncorrelated
    assert abs(np.vdot(a[0], c[0])) / a.shape[1] < 0.05
