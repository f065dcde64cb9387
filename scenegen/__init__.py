"""Seeded synthetic scenes shared by the FP64 oracle and the HIP library.

This module only builds meshes, boundary masks and seeded random state.  It
holds none of the method's arithmetic: no Lame conversion, no rest-shape
precomputation, no masses, no energies.  Both sides receive the same arrays
bit for bit and derive everything else on their own.

The paper measures on its own scenes (stretched cube, twisted beam, cloth);
their meshes are not public, so procedural grids of the same kind stand in
(Sec. 7, Tables 2-3).  Grid conventions:

* Tet grids: box of nx*ny*nz cubes of edge h, node id i + (nx+1)(j + (ny+1)k),
  cube id i + nx(j + ny k), element id 6*cube + p where p indexes the
  permutations of the axes in lexicographic order (Kuhn/Freudenthal split:
  the tet follows the path v000 -> +e_p0 -> +e_p1 -> v111).  Tets of odd
  permutations have vertices 2 and 3 swapped so that every tet is positively
  oriented; this is decided from the permutation parity, not from geometry.
* Quadratic tet grids: the tet grid's nodes keep their ids; every distinct
  tet edge (i, j), i < j, gets a mid-edge node at the midpoint of its rest
  endpoints, numbered after the vertices in ascending (i, j) order.  Element
  connectivity is (4 corners, 6 edge nodes) in the App. A order above.
* Cubic tet grids: vertices keep their ids; every distinct edge (i, j), i < j,
  gets the nodes at 1/3 and 2/3 from i (numbered in that order, edges in
  ascending (i, j)), then every distinct face (i < j < k) a node at its
  centroid (faces in ascending order).
* Cloth grids: m*m cells on [0,size]^2 at height z0, node id i + (m+1)j, each
  cell split along (i,j)->(i+1,j+1) into two counter-clockwise triangles.
  Hinges are the interior edges shared by two triangles, listed as
  (edge v0, edge v1, opposite vertex of the first triangle, opposite vertex of
  the second triangle), ordered by (min, max) edge node ids.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

SNH_TET4 = 0
STVK_TRI3 = 1
HINGE4 = 2
NH_TET4 = 3
STVK_TET4 = 4
FCR_TET4 = 5
ARAP_TET4 = 6
SNH_TET10 = 7
SNH_TET20 = 8

NODES_PER_ELEM = {SNH_TET4: 4, STVK_TRI3: 3, HINGE4: 4, NH_TET4: 4, STVK_TET4: 4, FCR_TET4: 4,
                  ARAP_TET4: 4, SNH_TET10: 10, SNH_TET20: 20}

# Quadratic tet node order (App. A, tet10 interpolation): corners 0-3, then the
# mid-edge nodes of edges (0,1), (1,2), (2,0), (0,3), (1,3), (2,3).
TET10_EDGES = ((0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3))
# Cubic tet node order: corners 0-3; for edge k = (i, j) of the list above the
# nodes 4 + 2k (one third from i) and 5 + 2k (one third from j); the face
# nodes 16 + c (centroid of the face opposite corner c).

_PERMS = list(itertools.permutations(range(3)))          # lexicographic order
_PERM_ODD = [False, True, True, False, False, True]      # parity of each entry


@dataclass
class EnergySet:
    """One energy applied to a set of elements (the element set of Eq. 5)."""
    kind: int
    conn: np.ndarray                   # (n_elem, k) int32
    young: float = 1e5                 # Young's modulus when per-element is None
    young_per_elem: np.ndarray | None = None   # (n_elem,) float64 or None
    poisson: float = 0.4
    thickness: float = 1.0             # membrane thickness (tri only)
    bend_kb: float = 0.0               # bending stiffness (hinge only)
    density: float = 1000.0            # kg/m^3 (tets and membranes)


@dataclass
class ContactList:
    """Candidate contacts of the point-plane barrier: node p against the plane
    of nodes t0, t1, t2 (rows (p, t0, t1, t2)); barrier stiffness and range."""
    tuples: np.ndarray                 # (n, 4) int32
    kc: float = 1e3
    dhat: float = 1e-3


@dataclass
class Scene:
    name: str
    X: np.ndarray                      # (N,3) float64 rest positions
    energies: list[EnergySet]
    fixed: np.ndarray                  # (N,) uint8, 1 = Dirichlet node
    x0: np.ndarray                     # (N,3) float64 positions x(t)
    v0: np.ndarray                     # (N,3) float64 velocities v(t)
    dt: float = 0.01
    gravity: tuple = (0.0, 0.0, -9.81)
    meta: dict = field(default_factory=dict)
    contacts: ContactList | None = None

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    def n_elements(self) -> int:
        return int(sum(e.conn.shape[0] for e in self.energies))


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------
def tet_grid(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)):
    """Regular box of nx*ny*nz cubes, each split into 6 positively oriented tets."""
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                             indexing="ij")
    # node id = i + (nx+1)(j + (ny+1)k): order the flattened arrays accordingly
    X = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                  kk.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64) * h
    X += np.asarray(origin, dtype=np.float64)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    ncube = ci.size
    tets = np.empty((ncube, 6, 4), dtype=np.int64)
    unit = np.eye(3, dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        pos = np.zeros(3, dtype=np.int64)
        path = [pos.copy()]
        for ax in perm:
            pos = pos + unit[ax]
            path.append(pos.copy())
        verts = [nid(ci + o[0], cj + o[1], ck + o[2]) for o in path]
        if _PERM_ODD[p]:
            verts[2], verts[3] = verts[3], verts[2]
        for a in range(4):
            tets[:, p, a] = verts[a]
    return X, tets.reshape(-1, 4).astype(np.int32)


def tet10_grid(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)):
    """The tet grid with a mid-edge node on every tet edge (quadratic tets)."""
    X, tets = tet_grid(nx, ny, nz, h, origin)
    nv = X.shape[0]
    t = tets.astype(np.int64)
    ends = np.stack([np.stack([t[:, i], t[:, j]], axis=1) for i, j in TET10_EDGES], axis=1)
    lo = ends.min(axis=2)
    hi = ends.max(axis=2)
    key = lo * nv + hi                                    # (n_tet, 6)
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    ulo, uhi = uniq // nv, uniq % nv
    Xe = 0.5 * (X[ulo] + X[uhi])
    conn = np.concatenate([t, nv + inv.reshape(-1, 6)], axis=1)
    return np.concatenate([X, Xe]), conn.astype(np.int32)


def tet20_grid(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)):
    """The tet grid with two nodes on every tet edge and one on every face
    (cubic tets)."""
    X, tets = tet_grid(nx, ny, nz, h, origin)
    nv = X.shape[0]
    t = tets.astype(np.int64)
    ends = np.stack([np.stack([t[:, i], t[:, j]], axis=1) for i, j in TET10_EDGES], axis=1)
    lo, hi = ends.min(axis=2), ends.max(axis=2)
    ekey = lo * nv + hi
    uniq, inv = np.unique(ekey.ravel(), return_inverse=True)
    inv = inv.reshape(-1, 6)
    ulo, uhi = uniq // nv, uniq % nv
    Xe = np.empty((2 * uniq.size, 3))
    Xe[0::2] = (2.0 * X[ulo] + X[uhi]) / 3.0
    Xe[1::2] = (X[ulo] + 2.0 * X[uhi]) / 3.0
    # element edge nodes: the one nearer the element's first endpoint first
    first_is_lo = ends[:, :, 0] == lo
    near_i = nv + 2 * inv + np.where(first_is_lo, 0, 1)
    near_j = nv + 2 * inv + np.where(first_is_lo, 1, 0)
    faces = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]       # opposite corner c
    fv = np.sort(np.stack([t[:, list(f)] for f in faces], axis=1), axis=2)   # (n, 4, 3)
    fkey = (fv[:, :, 0] * nv + fv[:, :, 1]) * nv + fv[:, :, 2]
    funiq, finv = np.unique(fkey.ravel(), return_inverse=True)
    f0 = funiq // (nv * nv)
    f1 = (funiq // nv) % nv
    f2 = funiq % nv
    Xf = (X[f0] + X[f1] + X[f2]) / 3.0
    nf0 = nv + 2 * uniq.size
    conn = np.concatenate([t, np.stack([near_i, near_j], axis=2).reshape(-1, 12),
                           nf0 + finv.reshape(-1, 4)], axis=1)
    return np.concatenate([X, Xe, Xf]), conn.astype(np.int32)


def cloth_grid(m: int, size: float = 1.0, z0: float = 0.0, origin_xy=(0.0, 0.0)):
    """m*m cells on [0,size]^2 at height z0, two counter-clockwise triangles per cell."""
    jj, ii = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    step = size / m
    X = np.stack([ii.ravel() * step + origin_xy[0], jj.ravel() * step + origin_xy[1],
                  np.full(ii.size, z0)], axis=1).astype(np.float64)

    def nid(i, j):
        return i + (m + 1) * j

    cj, ci = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    v00, v10 = nid(ci, cj), nid(ci + 1, cj)
    v01, v11 = nid(ci, cj + 1), nid(ci + 1, cj + 1)
    tris = np.empty((ci.size, 2, 3), dtype=np.int64)
    tris[:, 0] = np.stack([v00, v10, v11], axis=1)
    tris[:, 1] = np.stack([v00, v11, v01], axis=1)
    return X, tris.reshape(-1, 3).astype(np.int32)


def hinges_from_triangles(tris: np.ndarray) -> np.ndarray:
    """Interior edges shared by exactly two triangles -> (e0, e1, opp_a, opp_b)."""
    t = np.asarray(tris, dtype=np.int64)
    nt = t.shape[0]
    # each triangle edge (local a,b) with opposite vertex c
    loc = [(0, 1, 2), (1, 2, 0), (2, 0, 1)]
    ea = np.concatenate([t[:, a] for a, _, _ in loc])
    eb = np.concatenate([t[:, b] for _, b, _ in loc])
    opp = np.concatenate([t[:, c] for _, _, c in loc])
    tri_id = np.concatenate([np.arange(nt)] * 3)
    lo = np.minimum(ea, eb)
    hi = np.maximum(ea, eb)
    order = np.lexsort((tri_id, hi, lo))
    lo, hi, opp, tri_id = lo[order], hi[order], opp[order], tri_id[order]
    same = (lo[:-1] == lo[1:]) & (hi[:-1] == hi[1:])
    if np.any(same[:-1] & same[1:]):
        raise ValueError("non-manifold edge (shared by more than two triangles)")
    first = np.nonzero(same)[0]
    hinges = np.stack([lo[first], hi[first], opp[first], opp[first + 1]], axis=1)
    return hinges.astype(np.int32)


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------
def _bottom_fixed(X: np.ndarray, z_min: float | None = None) -> np.ndarray:
    z = X[:, 2]
    zmin = z.min() if z_min is None else z_min
    return (np.abs(z - zmin) <= 1e-12).astype(np.uint8)


def _grid_for(kind):
    return {SNH_TET10: tet10_grid, SNH_TET20: tet20_grid}.get(kind, tet_grid)


def tet_cube_scene(n: int, h: float = 0.01, young: float = 1e5, poisson: float = 0.4,
                   density: float = 1000.0, dt: float = 0.01, seed: int = 1,
                   perturb: float = 0.01, vel_std: float = 0.0, name: str | None = None,
                   dims: tuple | None = None, kind: int = SNH_TET4) -> Scene:
    """Cube (or box, via dims) of 6-tet cubes with the bottom face fixed.

    x(t) = X + U(-perturb*h, perturb*h)^3 on free nodes; v(t) ~ N(0, vel_std^2)
    on free nodes.  Draw order: perturbations (node-major), then velocities.
    kind: the tet material (SNH_TET4, NH_TET4, STVK_TET4, FCR_TET4, ARAP_TET4),
    or SNH_TET10 for quadratic Stable Neo-Hookean tets on the same cubes.
    """
    nx, ny, nz = dims if dims is not None else (n, n, n)
    X, tets = _grid_for(kind)(nx, ny, nz, h)
    fixed = _bottom_fixed(X)
    rng = np.random.default_rng(seed)
    N = X.shape[0]
    pert = rng.uniform(-perturb * h, perturb * h, size=(N, 3)) if perturb > 0 else np.zeros((N, 3))
    vel = rng.normal(0.0, vel_std, size=(N, 3)) if vel_std > 0 else np.zeros((N, 3))
    free = (fixed == 0)[:, None]
    x0 = X + np.where(free, pert, 0.0)
    v0 = np.where(free, vel, 0.0)
    es = EnergySet(kind, tets, young=young, poisson=poisson, density=density)
    return Scene(name or f"tetcube{nx}x{ny}x{nz}", X, [es], fixed, x0, v0, dt=dt,
                 meta=dict(n=n, h=h, seed=seed))


def stretched_box_scene(kind: int, dims: tuple = (40, 40, 60), h: float = 0.01,
                        young: float = 1e4, poisson: float = 0.3, stretch: float = 0.2,
                        seed: int = 6) -> Scene:
    """The material comparison workload (Sec. 6.1, Table 3): a box of 6-tet
    cubes (40 x 40 x 60 cubes: 41*41*61 nodes = 307,623 DoF), E=1e4 Pa,
    nu=0.3, bottom face fixed, top face fixed at (1 + stretch) of the height,
    interior stretched affinely in z plus +-1% noise (seed).  SNH_TET10
    builds the same box from quadratic tets."""
    nx, ny, nz = dims
    X, tets = _grid_for(kind)(nx, ny, nz, h)
    z = X[:, 2]
    top = z >= z.max() - 1e-12
    fixed = (_bottom_fixed(X).astype(bool) | top).astype(np.uint8)
    rng = np.random.default_rng(seed)
    pert = rng.uniform(-0.01 * h, 0.01 * h, size=X.shape)
    x0 = X.copy()
    x0[:, 2] *= 1.0 + stretch
    x0 = np.where(fixed[:, None] == 1, x0, x0 + pert)
    es = EnergySet(kind, tets, young=young, poisson=poisson, density=1000.0)
    return Scene(f"stretched-box-k{kind}", X, [es], fixed, x0, np.zeros_like(X), dt=0.01,
                 meta=dict(dims=dims, h=h, stretch=stretch, seed=seed))


def contact_stack_scene(n: int = 4, h: float = 0.01, dhat: float = 1e-3, kc: float = 1e3,
                        gap: float = 1.0, noise: float = 0.5, vz: float = -0.05,
                        seed: int = 9, neighbors: bool = False) -> Scene:
    """Two SNH cubes of n^3 6-tet cubes, the upper one resting gap * dhat above
    the lower one's top face (bottom face of the lower cube fixed).  Upper
    nodes get a vertical offset U(-noise, noise) * dhat and velocity vz.
    Candidate contacts: every node of the upper cube's bottom face against the
    lower top-face triangle (v00, v10, v11) of the cell below it, so about
    half of them are within d_hat.  neighbors=True lists instead both
    triangles of every cell touching the node's position (up to 8 per node),
    the candidate set of a proximity query with a one-cell margin."""
    X1, t1 = tet_grid(n, n, n, h)
    X2, t2 = tet_grid(n, n, n, h, origin=(0.0, 0.0, n * h + gap * dhat))
    N1 = X1.shape[0]
    X = np.concatenate([X1, X2])
    tets = np.concatenate([t1, t2 + N1]).astype(np.int32)
    fixed = np.concatenate([_bottom_fixed(X1), np.zeros(N1, np.uint8)])
    rng = np.random.default_rng(seed)
    x0 = X.copy()
    x0[N1:, 2] += rng.uniform(-noise, noise, N1) * dhat
    v0 = np.zeros_like(X)
    v0[N1:, 2] = vz

    def nid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)
    tuples = []
    for j in range(n + 1):
        for i in range(n + 1):
            if not neighbors:
                ci, cj = min(i, n - 1), min(j, n - 1)
                tuples.append([N1 + nid(i, j, 0), nid(ci, cj, n), nid(ci + 1, cj, n),
                               nid(ci + 1, cj + 1, n)])
                continue
            for cj in (j - 1, j):
                for ci in (i - 1, i):
                    if 0 <= ci < n and 0 <= cj < n:
                        v00, v10 = nid(ci, cj, n), nid(ci + 1, cj, n)
                        v01, v11 = nid(ci, cj + 1, n), nid(ci + 1, cj + 1, n)
                        tuples.append([N1 + nid(i, j, 0), v00, v10, v11])
                        tuples.append([N1 + nid(i, j, 0), v00, v11, v01])
    es = EnergySet(SNH_TET4, tets, young=1e5, poisson=0.4, density=1000.0)
    return Scene(f"contact-stack{n}", X, [es], fixed, x0, v0, dt=0.01,
                 meta=dict(n=n, h=h, gap=gap, noise=noise, seed=seed),
                 contacts=ContactList(np.asarray(tuples, dtype=np.int32), kc=kc, dhat=dhat))


def config_c1() -> Scene:
    """10^3 cubes, 6,000 tets, SNH E=1e5 nu=0.4, +-1% perturbation (seed 1), v=0."""
    return tet_cube_scene(10, h=0.01, young=1e5, poisson=0.4, seed=1, perturb=0.01,
                          vel_std=0.0, name="C1")


def config_c2(n: int = 64) -> Scene:
    """64^3 cubes, 1,572,864 tets, x(t)=X, v ~ N(0, 0.1^2) on free nodes (seed 2)."""
    return tet_cube_scene(n, h=0.01, young=1e5, poisson=0.4, seed=2, perturb=0.0,
                          vel_std=0.1, name="C2" if n == 64 else f"C2-n{n}")


def config_c4(n: int = 64) -> Scene:
    """C2 mesh, per-tet E ~ logU(1e4, 1e7) (seed 4), 30% compression, top+bottom fixed."""
    h = 0.01
    X, tets = tet_grid(n, n, n, h)
    rng = np.random.default_rng(4)
    young = np.exp(rng.uniform(np.log(1e4), np.log(1e7), size=tets.shape[0]))
    z = X[:, 2]
    top = np.abs(z - z.max()) <= 1e-12
    fixed = (_bottom_fixed(X).astype(bool) | top).astype(np.uint8)
    x0 = X.copy()
    x0[:, 2] *= 0.7
    es = EnergySet(SNH_TET4, tets, young_per_elem=young, poisson=0.4, density=1000.0)
    return Scene("C4" if n == 64 else f"C4-n{n}", X, [es], fixed, x0, np.zeros_like(X),
                 dt=0.01, meta=dict(n=n, h=h, seed=4))


def config_c3(m: int = 512, n_block: int = 32) -> Scene:
    """Cloth (StVK membrane + Bergou hinges) pinned along y=0, plus an SNH tet block.

    Cloth: [0,1]^2 at z0=1 m, E=1e4, nu=0.3, thickness 1e-3, rho=1000, k_b=1e-3.
    Block: n_block^3 cubes of 0.01 m at x>=2 m, bottom fixed.  The two are
    uncoupled; cloth nodes come first in the global numbering.
    """
    Xc, tris = cloth_grid(m, 1.0, z0=1.0)
    hinges = hinges_from_triangles(tris)
    Xb, tets = tet_grid(n_block, n_block, n_block, 0.01, origin=(2.0, 0.0, 0.0))
    nc = Xc.shape[0]
    X = np.concatenate([Xc, Xb])
    tets = tets + nc
    fixed = np.zeros(X.shape[0], dtype=np.uint8)
    fixed[:nc][np.abs(Xc[:, 1]) <= 1e-12] = 1
    fixed[nc:][np.abs(Xb[:, 2] - Xb[:, 2].min()) <= 1e-12] = 1
    es = [
        EnergySet(SNH_TET4, tets, young=1e5, poisson=0.4, density=1000.0),
        EnergySet(STVK_TRI3, tris, young=1e4, poisson=0.3, thickness=1e-3, density=1000.0),
        EnergySet(HINGE4, hinges, bend_kb=1e-3),
    ]
    return Scene("C3" if m == 512 else f"C3-m{m}", X, es, fixed, X.copy(), np.zeros_like(X),
                 dt=1.0 / 60.0, meta=dict(m=m, n_block=n_block, seed=3))


def cloth_scene(m: int, seed: int = 3, perturb: float = 0.0, kb: float = 1e-3) -> Scene:
    """Cloth only (membrane + hinges), pinned along y=0, optional seeded perturbation."""
    Xc, tris = cloth_grid(m, 1.0, z0=1.0)
    hinges = hinges_from_triangles(tris)
    fixed = (np.abs(Xc[:, 1]) <= 1e-12).astype(np.uint8)
    rng = np.random.default_rng(seed)
    h = 1.0 / m
    pert = rng.uniform(-perturb * h, perturb * h, size=Xc.shape) if perturb > 0 else 0.0
    x0 = Xc + np.where((fixed == 0)[:, None], pert, 0.0)
    es = [EnergySet(STVK_TRI3, tris, young=1e4, poisson=0.3, thickness=1e-3, density=1000.0),
          EnergySet(HINGE4, hinges, bend_kb=kb)]
    return Scene(f"cloth{m}", Xc, es, fixed, x0, np.zeros_like(Xc), dt=1.0 / 60.0,
                 meta=dict(m=m, seed=seed))


def config_c5_requests(n_requests: int = 256, rate: float = 200.0, seed: int = 5,
                       n_min: int = 8, n_max: int = 48):
    """Serving workload: Poisson arrivals, cube side n ~ round(logU(n_min, n_max)).

    Returns a list of dicts (arrival time [s], n, young, scene seed).  Each
    request's scene is built with tet_cube_scene(n, young=..., seed=...).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps)
    ns = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_requests))).astype(int)
    young = np.exp(rng.uniform(np.log(1e4), np.log(1e6), size=n_requests))
    seeds = rng.integers(0, 2**31 - 1, size=n_requests)
    return [dict(t=float(arrivals[i]), n=int(ns[i]), young=float(young[i]), seed=int(seeds[i]))
            for i in range(n_requests)]


def c5_request_scene(req: dict) -> Scene:
    return tet_cube_scene(req["n"], h=0.01, young=req["young"], poisson=0.4, seed=req["seed"],
                          perturb=0.01, vel_std=0.0, name=f"req-n{req['n']}")


def random_tets(n_elem: int, seed: int, inverted_frac: float = 0.2):
    """Stand-alone stressed tets for per-element tests: rest = random well-shaped
    tet, current = rest under a random affine map (some inverted, some compressed
    by 30%) plus noise.  Returns (x (E,4,3), X (E,4,3)); conn is implicit."""
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64) * 0.01
    X = base[None] + rng.uniform(-0.002, 0.002, size=(n_elem, 4, 3))
    A = np.eye(3)[None] + rng.uniform(-0.3, 0.3, size=(n_elem, 3, 3))
    flip = rng.uniform(size=n_elem) < inverted_frac
    A[flip, :, 2] *= -1.0
    comp = rng.uniform(size=n_elem) < 0.3
    A[comp] *= 0.7
    x = np.einsum("eij,eaj->eai", A, X) + rng.uniform(-1e-4, 1e-4, size=(n_elem, 4, 3))
    x += rng.uniform(-0.5, 0.5, size=(n_elem, 1, 3))
    return x, X
