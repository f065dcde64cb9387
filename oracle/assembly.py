"""Brute-force sparsity pattern, scatter map and assembly into 3x3 BSR (oracle).

TEST INFRASTRUCTURE ONLY.

* Pattern (Sec. 5.3, Eq. 11 and the BCRS paragraph): block (i, j) exists iff
  nodes i and j share an element of any energy, i = j included; every node has
  its diagonal block.  Rows hold ascending column indices; both triangles are
  stored.
* Scatter map (Alg. 1, GlobalIndex/BlockExists): entry (e, a, b) of an energy
  set is the BSR position of block (conn[e,a], conn[e,b]); local order is
  row-major over (a, b) in connectivity order.
* Assembly (Eq. 5 with the selection operators R_e, Alg. 1 AddInPlace): the
  global gradient is sum_e R_e^T g_e and the Hessian sum_e R_e^T H_e R_e, summed
  per block in energy-set order, then ascending element id; the inertia term of
  Eq. 2 is added last.
* Dirichlet nodes: gradient rows zero, Hessian rows and columns zero, identity
  diagonal block, applied after assembly so the pattern does not change.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import contact, elements
from .projection import project_psd
from .rest import lame, lumped_mass, young_array


def pattern(scene):
    """Return (row_ptr (N+1,), col_idx (nnzb,)) as int32 by brute force over pairs."""
    N = scene.n_nodes
    pairs = set((i, i) for i in range(N))
    for es in scene.energies:
        for elem in es.conn.tolist():
            for i in elem:
                for j in elem:
                    pairs.add((i, j))
    rows = [[] for _ in range(N)]
    for i, j in pairs:
        rows[i].append(j)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    col = []
    for i in range(N):
        r = sorted(rows[i])
        col.extend(r)
        row_ptr[i + 1] = row_ptr[i] + len(r)
    return row_ptr.astype(np.int32), np.asarray(col, dtype=np.int32)


def pattern_fast(scene):
    """Same pattern via numpy unique (used for large scenes; tested equal to pattern)."""
    N = scene.n_nodes
    keys = [np.arange(N, dtype=np.int64) * N + np.arange(N, dtype=np.int64)]
    for es in scene.energies:
        c = es.conn.astype(np.int64)
        k = c.shape[1]
        for a in range(k):
            for b in range(k):
                keys.append(c[:, a] * N + c[:, b])
    keys = np.unique(np.concatenate(keys))
    rows = keys // N
    cols = keys % N
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32)


def scatter_map(scene, row_ptr, col_idx):
    """List (one per energy set) of int32 arrays (n_elem, k, k) of BSR positions."""
    out = []
    for es in scene.energies:
        c = es.conn.astype(np.int64)
        n, k = c.shape
        smap = np.empty((n, k, k), dtype=np.int64)
        for a in range(k):
            for b in range(k):
                i = c[:, a]
                j = c[:, b]
                lo = row_ptr[i].astype(np.int64)
                hi = row_ptr[i + 1].astype(np.int64)
                # position of j inside row i: count of entries < j in the row
                pos = np.empty(n, dtype=np.int64)
                for e in range(n):
                    row = col_idx[lo[e]:hi[e]]
                    hit = np.nonzero(row == j[e])[0]
                    if hit.size != 1:
                        raise AssertionError("block missing from pattern")
                    pos[e] = lo[e] + hit[0]
                smap[:, a, b] = pos
        out.append(smap.astype(np.int32))
    return out


def assemble(scene, x, x_tilde=None, dt=None, project=False, dirichlet=True,
             want_hess=True, row_ptr=None, col_idx=None, x_lag=None):
    """Assemble E (float), g (N,3) and BSR values (nnzb,3,3) at positions x.

    Returns dict(E, g, row_ptr, col_idx, vals, E_parts).  With x_tilde/dt the
    inertia term of the incremental potential is included.  project=True
    replaces each element Hessian by its PSD projection before assembly;
    project="filter" instead filters the density Hessian of Stable
    Neo-Hookean tets (elements.snh_tet4_filtered) and projects the element
    Hessians of every other kind.
    x_lag: positions of the lagged rotations (default: rest).
    A scene with candidate contacts adds the conditional barrier (inactive
    candidates contribute nothing); its blocks are returned apart, as
    "contact_blocks" {(i, j): 3x3} (Dirichlet applied, element Hessians
    projected to PSD when project is set).
    """
    N = scene.n_nodes
    if row_ptr is None:
        row_ptr, col_idx = pattern_fast(scene)
    nnzb = col_idx.shape[0]
    lookup = {}
    g = np.zeros((N, 3))
    vals = np.zeros((nnzb, 3, 3)) if want_hess else None
    E_total = 0.0
    parts = []
    for es in scene.energies:
        Ee, ge, He = elements.element_eval(es, x, scene.X, want_hess, x_lag)
        filtered = want_hess and project == "filter" and es.kind == 0
        if filtered:
            mu, lam = lame(young_array(es), es.poisson)
            _, _, He = elements.snh_tet4_filtered(x[es.conn], scene.X[es.conn], mu, lam)
        parts.append(float(np.sum(Ee)))
        E_total += float(np.sum(Ee))
        c = es.conn
        k = c.shape[1]
        np.add.at(g, c.ravel(), ge.reshape(-1, 3))
        if want_hess:
            if project and not filtered:
                He = project_psd(He.reshape(-1, 3 * k, 3 * k)).reshape(He.shape)
            key = id(es)
            if key not in lookup:
                lookup[key] = _block_index(c, row_ptr, col_idx)
            pos = lookup[key]                                 # (n, k, k)
            blocks = He.transpose(0, 1, 3, 2, 4)             # (n, a, b, i, k)
            np.add.at(vals, pos.ravel(), blocks.reshape(-1, 3, 3))
    cblocks = {}
    cl = scene.contacts
    if cl is not None and cl.tuples.shape[0] > 0:
        Ec, gc, Hc, act = contact.point_plane_barrier(x[cl.tuples], cl.kc, cl.dhat, want_hess)
        parts.append(float(np.sum(Ec)))
        E_total += float(np.sum(Ec))
        np.add.at(g, cl.tuples.ravel(), gc.reshape(-1, 3))
        if want_hess:
            Ha = Hc[act].reshape(-1, 12, 12)
            if project:
                Ha = project_psd(Ha)
            Ha = Ha.reshape(-1, 4, 3, 4, 3)
            fixed = scene.fixed.astype(bool)
            for t, He in zip(cl.tuples[act], Ha):
                for a in range(4):
                    for b in range(4):
                        key = (int(t[a]), int(t[b]))
                        blk = He[a, :, b, :] if not (dirichlet and (fixed[t[a]] or fixed[t[b]])) \
                            else np.zeros((3, 3))
                        cblocks[key] = cblocks.get(key, np.zeros((3, 3))) + blk
    if x_tilde is not None:
        m = lumped_mass(scene)
        Ei, gi, w = elements.inertia(x, x_tilde, m, dt)
        parts.append(float(np.sum(Ei)))
        E_total += float(np.sum(Ei))
        g += gi
        if want_hess:
            diag = _diag_index(row_ptr, col_idx)
            vals[diag] += w[:, None, None] * np.eye(3)[None]
    if dirichlet:
        fixed = scene.fixed.astype(bool)
        g[fixed] = 0.0
        if want_hess:
            rows = np.repeat(np.arange(N), np.diff(row_ptr))
            kill = fixed[rows] | fixed[col_idx]
            vals[kill] = 0.0
            diag = _diag_index(row_ptr, col_idx)
            vals[diag[fixed]] = np.eye(3)
    return dict(E=E_total, g=g, row_ptr=row_ptr, col_idx=col_idx, vals=vals, E_parts=parts,
                contact_blocks=cblocks)


def _block_index(conn, row_ptr, col_idx):
    """Vectorised scatter-map lookup (equal to scatter_map; tested)."""
    c = conn.astype(np.int64)
    n, k = c.shape
    N = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(N, dtype=np.int64), np.diff(row_ptr))
    keys = rows * N + col_idx.astype(np.int64)          # sorted ascending
    want = c[:, :, None] * N + c[:, None, :]
    pos = np.searchsorted(keys, want)
    if not np.all(keys[np.minimum(pos, keys.size - 1)] == want):
        raise AssertionError("block missing from pattern")
    return pos


def _diag_index(row_ptr, col_idx):
    N = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    d = np.nonzero(rows == col_idx)[0]
    assert d.size == N
    return d


def energy(scene, x, x_tilde=None, dt=None, x_lag=None):
    """Total energy only (the line-search evaluation level)."""
    E = 0.0
    for es in scene.energies:
        Ee, _, _ = elements.element_eval(es, x, scene.X, want_hess=False, x_lag=x_lag)
        E += float(np.sum(Ee))
    cl = scene.contacts
    if cl is not None and cl.tuples.shape[0] > 0:
        Ec, _, _, _ = contact.point_plane_barrier(x[cl.tuples], cl.kc, cl.dhat, want_hess=False)
        E += float(np.sum(Ec))
    if x_tilde is not None:
        m = lumped_mass(scene)
        Ei, _, _ = elements.inertia(x, x_tilde, m, dt)
        E += float(np.sum(Ei))
    return E


def to_scipy(row_ptr, col_idx, vals, contact_blocks=None):
    """The assembled Hessian as a scipy CSR matrix, contact blocks added."""
    N = row_ptr.shape[0] - 1
    A = sp.bsr_matrix((vals, col_idx, row_ptr), shape=(3 * N, 3 * N)).tocsr()
    if contact_blocks:
        rows, cols, data = [], [], []
        for (i, j), b in contact_blocks.items():
            for r in range(3):
                for c in range(3):
                    rows.append(3 * i + r)
                    cols.append(3 * j + c)
                    data.append(b[r, c])
        A = A + sp.csr_matrix((data, (rows, cols)), shape=(3 * N, 3 * N))
    return A
