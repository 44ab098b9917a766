"""Seeded random vectors: right-hand sides, relaxation starts, gauge rotations."""
import numpy as np


def gaussian_vectors(count, length, seed, tag=0):
    """``count`` complex Gaussian vectors of ``length`` entries.

    Real and imaginary parts are independent N(0, 1).  ``(seed, tag)`` keys the
    stream, so right-hand sides (tag 0) and the starting vectors of each
    coarsening level (tag 1 + level) never share draws.  Returns complex128
    ``[count, length]``.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x6A55, int(tag)]))
    re = rng.standard_normal((int(count), int(length)))
    im = rng.standard_normal((int(count), int(length)))
    return re + 1j * im


def gauge_transform_field(volume, ncolor, seed):
    """Random local gauge rotation g(x): U(1) phases or Haar SU(3) matrices.

    Returns complex128 ``[site, ncolor, ncolor]``.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x6A06]))
    if ncolor == 1:
        return np.exp(1j * rng.uniform(-np.pi, np.pi, size=(volume, 1, 1)))
    Z = (rng.standard_normal((volume, ncolor, ncolor))
         + 1j * rng.standard_normal((volume, ncolor, ncolor))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q * np.exp(-1j * np.angle(det) / ncolor)[:, None, None]
