"""Material parameters and rest-shape quantities (oracle; test infrastructure).

* Lame parameters from Young's modulus and Poisson ratio: the standard 3D
  conversion (the paper states E and nu only, Sec. 6.1 / App. B).
* Stable Neo-Hookean re-parametrisation (App. B, Stable Neo-Hookean branch):
  mu' = 4/3 mu, lambda' = lambda + 5/6 mu.  The printed line is garbled (it
  applies 5/6 to lambda and uses integer-looking fractions); this is the reading
  under which the rest Hessian equals linear elasticity with the given (E, nu),
  which tests/test_oracle_pins.py checks against the textbook stiffness.
* Lumped masses for the inertia term of the incremental potential (Eq. 2):
  each tet gives rho*V/4 to its nodes, each membrane triangle rho*h*A/3.
  Quadratic tets (the paper does not say how their mass is lumped): HRZ
  lumping, the consistent mass diagonal rho int N_a^2 dV scaled to the total
  rho V.  With int L0^p L1^q L2^r L3^s dV = 6V p!q!r!s!/(p+q+r+s+3)! the
  diagonal is V/70 at a corner and 8V/105 at an edge node (sum 18V/35), so a
  corner gets rho V/36 and an edge node 4 rho V/27 (V of the straight-sided
  element, i.e. of its corner tet).  Cubic tets likewise: the diagonal is
  V/280 at a corner, 27V/1120 at an edge node and 27V/280 at a face node
  (sum 193V/280), so rho V/193, 27 rho V/772 and 27 rho V/193.
"""
from __future__ import annotations

import numpy as np


# Every tetrahedral element kind: Stable Neo-Hookean, classic Neo-Hookean,
# Saint Venant-Kirchhoff, fixed co-rotational, ARAP (scenegen numbering).
TET_KINDS = (0, 3, 4, 5, 6)
TET10_KIND = 7                     # quadratic Stable Neo-Hookean tet
TET20_KIND = 8                     # cubic Stable Neo-Hookean tet


def lame(young, poisson):
    """(mu, lambda) of isotropic linear elasticity."""
    young = np.asarray(young, dtype=np.float64)
    mu = young / (2.0 * (1.0 + poisson))
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    return mu, lam


def snh_reparam(mu, lam):
    """Stable Neo-Hookean (mu', lambda') from the linear-elasticity Lame pair."""
    return 4.0 / 3.0 * mu, lam + 5.0 / 6.0 * mu


def tet_volume(X):
    """|det Dm| / 6 for rest positions X of shape (E,4,3)."""
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return np.abs(np.linalg.det(Dm)) / 6.0


def tri_area(X):
    """Area of rest triangles X of shape (E,3,3)."""
    return 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1)


def lumped_mass(scene):
    """Per-node mass: sum over tets of rho V/4 and over triangles of rho h A/3."""
    m = np.zeros(scene.n_nodes)
    for es in scene.energies:
        if es.kind in TET_KINDS:
            V = tet_volume(scene.X[es.conn])
            np.add.at(m, es.conn.ravel(), np.repeat(es.density * V / 4.0, 4))
        elif es.kind in (TET10_KIND, TET20_KIND):
            V = tet_volume(scene.X[es.conn[:, :4]])
            if es.kind == TET10_KIND:
                share = np.array([1.0 / 36.0] * 4 + [4.0 / 27.0] * 6)
            else:
                share = np.array([1.0 / 193.0] * 4 + [27.0 / 772.0] * 12 + [27.0 / 193.0] * 4)
            np.add.at(m, es.conn.ravel(), (es.density * V[:, None] * share[None, :]).ravel())
        elif es.kind == 1:
            A = tri_area(scene.X[es.conn])
            np.add.at(m, es.conn.ravel(), np.repeat(es.density * es.thickness * A / 3.0, 3))
    return m


def young_array(es):
    n = es.conn.shape[0]
    if es.young_per_elem is not None:
        return np.asarray(es.young_per_elem, dtype=np.float64)
    return np.full(n, float(es.young))
