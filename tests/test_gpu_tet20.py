"""Cubic Stable Neo-Hookean tets (20 nodes, Eq. 12 with Keast's 11-point rule)
on the HIP path, through the C-ABI, against the float64 oracle.

Tolerances as elsewhere: normwise 1e-10 in float64, 1e-4 in float32.  The
pattern and scatter map are compared exactly, the masses to rounding.  The
device relabels each element so that the evaluated node is node 0 (corner), 4
(edge node) or 19 (face node), and lists the rule's points in its own order,
so the two sides differ by rounding only.  Interior corners of the boxes
belong to 24 elements: their row batches hold more than 256 / 11 incidences
and take two evaluation passes.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements, newton, rest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL = 1e-4
EDGES = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]
FACES = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


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


def _scene(n=3, seed=81, perturb=0.05, vel=0.05):
    return sg.tet_cube_scene(n, kind=sg.SNH_TET20, seed=seed, perturb=perturb, vel_std=vel)


def _bsr(vals):
    return vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3)


def _cubic_nodes(P):
    """The 20 nodes of straight-sided cubic tets from their corners (E,4,3)."""
    e = []
    for i, j in EDGES:
        e += [(2 * P[:, i] + P[:, j]) / 3, (P[:, i] + 2 * P[:, j]) / 3]
    f = [P[:, list(c)].mean(1) for c in FACES]
    return np.concatenate([P, np.stack(e, 1), np.stack(f, 1)], 1)


def test_tet20_pattern_scatter_and_masses(symx):
    scene = _scene()
    mesh = symx.Mesh(scene)
    rp, ci, maps = mesh.pattern()
    rp_o, ci_o = assembly.pattern_fast(scene)
    assert np.array_equal(rp, rp_o)
    assert np.array_equal(ci, ci_o)
    assert np.array_equal(maps[0], assembly._block_index(scene.energies[0].conn, rp_o, ci_o))
    assert rel(mesh.masses(), rest.lumped_mass(scene)) < 1e-14
    assert np.bincount(scene.energies[0].conn.ravel()).max() == 24
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tet20_elem_derivatives(symx, precision):
    """Curved, stretched and compressed cubic elements (a disjoint set)."""
    n = 200
    rng = np.random.default_rng(82)
    x4, X4 = sg.random_tets(n, 83, inverted_frac=0.0)
    X = _cubic_nodes(X4)
    x = _cubic_nodes(x4) + rng.uniform(-4e-4, 4e-4, (n, 20, 3))
    conn = np.arange(20 * n, dtype=np.int32).reshape(n, 20)
    es = sg.EnergySet(sg.SNH_TET20, conn, young_per_elem=np.exp(rng.uniform(np.log(1e4),
                                                                               np.log(1e7), n)),
                      poisson=0.4)
    Xf, xf = X.reshape(-1, 3), x.reshape(-1, 3)
    scene = sg.Scene("loose20", Xf, [es], np.zeros(Xf.shape[0], np.uint8), xf, np.zeros_like(Xf))
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    E, g, H = mesh.eval_derivatives(0, xf, precision=p)
    Eo, go, Ho = elements.element_eval(es, xf, Xf)
    assert rel(E.cpu().numpy(), Eo) < tol
    assert rel(g.cpu().numpy().reshape(n, 20, 3), go) < tol
    Hd = H.cpu().numpy().reshape(n, 60, 60)
    Hr = Ho.reshape(n, 60, 60)
    assert max(rel(Hd[e], Hr[e]) for e in range(n)) < tol
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tet20_assembly(symx, precision):
    scene = _scene(3, seed=84, perturb=0.08)
    mesh = symx.Mesh(scene)
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    E, g, vals = mesh.assemble(scene.x0, xt, dt, flags, p)
    ref = assembly.assemble(scene, scene.x0, xt, dt)
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < tol
    assert rel(_bsr(vals), ref["vals"]) < tol
    g2 = mesh.assemble(scene.x0, xt, dt, symx.SYMX_EVAL_GRAD | symx.SYMX_DIRICHLET, p)[1]
    assert rel(g2.cpu().numpy(), ref["g"]) < tol
    # elastic only, no Dirichlet
    E3, g3, v3 = mesh.assemble(scene.x0, None, 0.0,
                               symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS, p)
    ref3 = assembly.assemble(scene, scene.x0, dirichlet=False)
    assert abs(E3 - ref3["E"]) <= tol * abs(ref3["E"])
    assert rel(g3.cpu().numpy(), ref3["g"]) < tol
    assert rel(_bsr(v3), ref3["vals"]) < tol
    mesh.close()


def test_tet20_assembly_bitwise_reproducible(symx):
    scene = _scene(3, seed=85)
    mesh = symx.Mesh(scene)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
    a = mesh.assemble(scene.x0, None, 0.0, flags, symx.SYMX_F32)
    b = mesh.assemble(scene.x0, None, 0.0, flags, symx.SYMX_F32)
    assert a[0] == b[0]
    assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_tet20_newton_step(symx, precision):
    """A stretched cubic box, one implicit-Euler step: the oracle's float64
    gradient at the device's answer meets the tolerance and the minimiser is
    the oracle's own Newton step's."""
    scene = sg.stretched_box_scene(sg.SNH_TET20, dims=(2, 2, 3))
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=scene.dt, precision=p))
    mesh.close()
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xh = x.cpu().numpy()
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, dt, want_hess=False)["g"])
    assert rep.residual0 == pytest.approx(r0, rel=1e-10)
    g = assembly.assemble(scene, xh, xt, dt, want_hess=False)["g"]
    assert np.linalg.norm(g) <= 1.01e-6 * r0
    ok, xo, repo = newton.newton_solve(scene, scene.x0, scene.v0, dt, newton.StepParams(dt=dt))
    assert ok
    m_min = rest.lumped_mass(scene).min()
    assert np.max(np.abs(xh - xo)) <= 2.0e-6 * r0 * dt * dt / m_min
    assert rep.energy == pytest.approx(repo["energy"], rel=1e-9)


def test_tet20_rejections(symx):
    """No projection for cubic tets; a cubic set shares a mesh with no other
    set (linear or quadratic); no contacts on such a mesh."""
    scene = _scene(2)
    mesh = symx.Mesh(scene)
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
             | symx.SYMX_PROJECT_PSD)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.assemble(scene.x0, None, 0.0, flags, symx.SYMX_F64)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.eval_derivatives(0, scene.x0, flags=flags)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contacts(np.array([[0, 1, 2, 3]], dtype=np.int32), 1e3, 1e-3)
    mesh.close()
    N = scene.n_nodes
    for other in (sg.tet_cube_scene(2), sg.tet_cube_scene(2, kind=sg.SNH_TET10)):
        es = [scene.energies[0], sg.EnergySet(other.energies[0].kind, other.energies[0].conn + N)]
        mixed = sg.Scene("mixed", np.concatenate([scene.X, other.X + 0.1]), es,
                         np.concatenate([scene.fixed, other.fixed]),
                         np.concatenate([scene.x0, other.x0 + 0.1]),
                         np.zeros((N + other.n_nodes, 3)))
        with pytest.raises(symx.SymxError, match="INVALID_ARG"):
            symx.Mesh(mixed)


def test_tet20_crowded_node_rejected(symx):
    """A row batch holds at most 32 cubic incidences: a node shared by 33
    elements is an argument error that names the limit."""
    n = 33
    _, X4 = sg.random_tets(n, 86, inverted_frac=0.0)
    X4 = X4 - X4[:, :1]                                  # corner 0 of every element at 0
    X = _cubic_nodes(X4).reshape(-1, 3)
    conn = np.arange(20 * n, dtype=np.int32).reshape(n, 20)
    conn[:, 0] = 0                                       # corner 0 shared by all
    es = sg.EnergySet(sg.SNH_TET20, conn, young=1e5, poisson=0.4)
    scene = sg.Scene("fan20", X, [es], np.zeros(X.shape[0], np.uint8), X.copy(), np.zeros_like(X))
    with pytest.raises(symx.SymxError, match="INVALID_ARG.*more than 32 elements"):
        symx.Mesh(scene)
