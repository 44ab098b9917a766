"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package generates inputs only: gauge configurations (quenched compact U(1)
by heatbath, smooth random SU(3) fields), Gaussian right-hand sides and the
random starting vectors of the near-null-vector relaxation.  It holds none of
the multigrid method's arithmetic; the oracle and the GPU library both consume
what it produces and share nothing else.

Lattice conventions used by every generator here:
  * a d-dimensional lattice of extents ``dims = (L_1, ..., L_d)``, site index
    ``x_1 + L_1*(x_2 + L_2*(...))`` (x_1 fastest, time = last axis);
  * a gauge field is a complex128 array ``U[mu, site, a, b]`` with ``a, b`` the
    colour indices (``ncolor = 1`` for U(1));
  * a fermion vector is complex128 ``[site, colour]`` (flattened).
"""
from .gauge import (u1_heatbath, u1_plaquette, su3_smooth_random,
                    su3_plaquette, unit_gauge, config_seed)
from .vectors import gaussian_vectors, gauge_transform_field

__all__ = ["u1_heatbath", "u1_plaquette", "su3_smooth_random", "su3_plaquette",
           "unit_gauge", "config_seed", "gaussian_vectors",
           "gauge_transform_field"]
