"""Dynamic topology (Sec. 5.2; Alg. 1's rebuild of the sparsity when it
changes): a dynamic element set replaced between steps, through the C-ABI,
against the float64 oracle.

The device keeps the static sets' block pattern and puts the dynamic
elements' couplings in a second block matrix built on the device; the
oracle holds the same elements as one more energy set of the scene (its last
set), so its blocks are the sums of the device's two matrices.  Tolerances:
normwise 1e-10 in float64, 1e-4 in float32.
"""
import dataclasses

import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements, newton, rest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL = 1e-4
FLAGS = 1 | 2 | 4 | 16   # E, gradient, Hessian, Dirichlet


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def symx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02156_amd import symx as s
    s.load()
    return s


def _split(seed=31, perturb=0.1, n=4):
    """A tet box whose elements are split into a static set (kept by the mesh)
    and a pool of candidate dynamic elements (stiffer, other material)."""
    s = sg.tet_cube_scene(n, seed=seed, perturb=perturb)
    conn = s.energies[0].conn
    rng = np.random.default_rng(seed)
    dyn_ids = np.sort(rng.choice(conn.shape[0], conn.shape[0] // 3, replace=False))
    keep = np.setdiff1d(np.arange(conn.shape[0]), dyn_ids)
    static = dataclasses.replace(s, energies=[dataclasses.replace(s.energies[0], conn=conn[keep])])
    pool = conn[dyn_ids]
    return static, pool


def _dyn_set(kind, conn, seed):
    rng = np.random.default_rng(seed)
    return sg.EnergySet(kind, np.ascontiguousarray(conn, dtype=np.int32),
                        young_per_elem=np.exp(rng.uniform(np.log(5e4), np.log(5e5), conn.shape[0])),
                        poisson=0.35, density=800.0)


def _with(static, dyn):
    """The oracle's scene: the static sets and, last, the dynamic set."""
    return dataclasses.replace(static, energies=list(static.energies) + ([dyn] if dyn is not None
                                                                         and dyn.conn.shape[0]
                                                                         else []))


def _blocks(rp, ci, vals):
    out = {}
    for i in range(len(rp) - 1):
        for q in range(rp[i], rp[i + 1]):
            out[(i, int(ci[q]))] = vals[q]
    return out


def _check(symx, mesh, static, dyn, precision, x=None):
    full = _with(static, dyn)
    x = full.x0 if x is None else x
    xt = elements.x_tilde(full.x0, full.v0, full.dt, full.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    E, g, vals = mesh.assemble(x, xt, full.dt, FLAGS, p)
    ref = assembly.assemble(full, x, xt, full.dt)
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < tol
    assert rel(mesh.masses(), rest.lumped_mass(full)) < 1e-14
    rp, ci, _ = mesh.pattern()
    dev = _blocks(rp, ci, vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3))
    drp, dci, dvals = mesh.contact_bsr(p)
    for key, b in _blocks(drp, dci, dvals).items():
        dev[key] = dev.get(key, np.zeros((3, 3))) + b
    want = _blocks(ref["row_ptr"], ref["col_idx"], ref["vals"])
    assert set(want) <= set(dev)
    scale = max(np.abs(b).max() for b in want.values())
    err = max(np.abs(dev[k] - want.get(k, np.zeros((3, 3)))).max() for k in dev)
    assert err <= tol * scale


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dynamic_set_assembly(symx, precision):
    """A third of a box's tets as a dynamic set of another material: energy,
    gradient, masses and the sum of the two block matrices match the oracle
    holding them as one more set."""
    static, pool = _split()
    dyn = _dyn_set(sg.SNH_TET4, pool, 1)
    mesh = symx.Mesh(static)
    mesh.set_dynamic_elements(dyn)
    _check(symx, mesh, static, dyn, precision)
    mesh.close()


def test_dynamic_set_changes(symx):
    """Replace the set (fewer elements, other elements, another kind, more
    elements than the first list held), then remove it; every state matches
    the oracle, and removal restores the static masses and matrix."""
    static, pool = _split(seed=32)
    mesh = symx.Mesh(static)
    rng = np.random.default_rng(5)
    lists = [
        _dyn_set(sg.SNH_TET4, pool, 2),
        _dyn_set(sg.SNH_TET4, pool[: len(pool) // 3], 3),
        _dyn_set(sg.NH_TET4, pool[rng.permutation(len(pool))[: len(pool) // 2]], 4),
        _dyn_set(sg.STVK_TET4, np.concatenate([pool, static.energies[0].conn[:20]]), 5),
    ]
    for dyn in lists:
        mesh.set_dynamic_elements(dyn)
        _check(symx, mesh, static, dyn, "f64")
    mesh.set_dynamic_elements(None)
    _check(symx, mesh, static, None, "f64")
    assert mesh.contact_bsr(symx.SYMX_F64)[1].size == 0
    mesh.close()


def test_dynamic_hinges_on_cloth(symx):
    """Bending hinges as the dynamic set of a cloth's membranes (no mass)."""
    c = sg.cloth_scene(5, perturb=0.2)
    static = dataclasses.replace(c, energies=[c.energies[0]])
    hinges = c.energies[1]
    mesh = symx.Mesh(static)
    mesh.set_dynamic_elements(hinges)
    for precision in ("f64", "f32"):
        _check(symx, mesh, static, hinges, precision)
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_dynamic_set_newton_step(symx, precision):
    """One implicit-Euler step with a dynamic set reaches the oracle's
    minimiser of the scene holding it as a set."""
    static, pool = _split(seed=33, perturb=0.2)
    dyn = _dyn_set(sg.SNH_TET4, pool, 6)
    full = _with(static, dyn)
    mesh = symx.Mesh(static)
    mesh.set_dynamic_elements(dyn)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    x = torch.tensor(full.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(full.v0, dtype=torch.float64, device="cuda")
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=full.dt, precision=p))
    mesh.close()
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xh = x.cpu().numpy()
    dt = full.dt
    xt = elements.x_tilde(full.x0, full.v0, dt, full.gravity)
    r0 = np.linalg.norm(assembly.assemble(full, full.x0, xt, dt, want_hess=False)["g"])
    assert rep.residual0 == pytest.approx(r0, rel=1e-10)
    assert np.linalg.norm(assembly.assemble(full, xh, xt, dt, want_hess=False)["g"]) <= 1.01e-6 * r0
    ok, xo, repo = newton.newton_solve(full, full.x0, full.v0, dt, newton.StepParams(dt=dt))
    assert ok
    m_min = rest.lumped_mass(full).min()
    assert np.max(np.abs(xh - xo)) <= 2.0e-6 * r0 * dt * dt / m_min
    assert rep.energy == pytest.approx(repo["energy"], rel=1e-9)


def test_dynamic_set_rejections(symx):
    static, pool = _split(seed=34)
    mesh = symx.Mesh(static)
    bad = _dyn_set(sg.SNH_TET4, pool.copy(), 7)
    bad.conn[0, 1] = bad.conn[0, 0]
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_dynamic_elements(bad)
    bad = _dyn_set(sg.SNH_TET4, pool.copy(), 7)
    bad.conn[1, 2] = static.n_nodes
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_dynamic_elements(bad)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_dynamic_elements(_dyn_set(sg.FCR_TET4, pool, 7))
    # a mesh holds contacts or a dynamic set, not both
    mesh.set_dynamic_elements(_dyn_set(sg.SNH_TET4, pool, 8))
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contacts(pool[:4], 1e3, 1e-3)
    mesh.set_dynamic_elements(None)
    mesh.set_contacts(pool[:4], 1e3, 1e-3)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_dynamic_elements(_dyn_set(sg.SNH_TET4, pool, 8))
    mesh.close()
