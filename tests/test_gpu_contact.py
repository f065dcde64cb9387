"""The conditional point-plane contact barrier (Eq. 9 activation, the contact
potential of Sec. 5.4) and the dynamic contact pattern, on the HIP path
through the C-ABI, against the float64 oracle.

The device keeps the mesh's block pattern and puts the couplings of the
candidate contacts in a second block matrix (blocks of inactive candidates
zero); the oracle returns the active contact blocks apart.  Tolerances:
normwise 1e-10 in float64, 1e-4 in float32.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, contact, elements, newton, rest

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


def _bsr(vals):
    return vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3)


def _all_triangles(scene, n):
    """Every upper bottom-face node against every lower top-face triangle
    (two per cell): many candidates, the same planes, mixed activity."""
    N1 = (n + 1) ** 3

    def nid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)
    tris = []
    for cj in range(n):
        for ci in range(n):
            v00, v10 = nid(ci, cj, n), nid(ci + 1, cj, n)
            v01, v11 = nid(ci, cj + 1, n), nid(ci + 1, cj + 1, n)
            tris += [(v00, v10, v11), (v00, v11, v01)]
    pts = [N1 + nid(i, j, 0) for j in range(n + 1) for i in range(n + 1)]
    return np.array([[p, *t] for p in pts for t in tris], dtype=np.int32)


def _expected_pattern(tuples, n_nodes):
    """Row pointers and sorted columns of every node pair of every candidate
    (diagonal included): the contact pattern, written out with numpy."""
    t = np.asarray(tuples, dtype=np.int64)
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    key = np.unique(rows * n_nodes + cols)
    r, c = key // n_nodes, key % n_nodes
    rp = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), c


def _check_contact_blocks(mesh, ref, precision, tol):
    rp, ci, vals = mesh.contact_bsr(precision)
    scale = max(np.abs(b).max() for b in ref["contact_blocks"].values())
    seen = set()
    err = 0.0
    for i in range(len(rp) - 1):
        for p in range(rp[i], rp[i + 1]):
            key = (i, int(ci[p]))
            seen.add(key)
            want = ref["contact_blocks"].get(key, np.zeros((3, 3)))
            err = max(err, np.abs(vals[p] - want).max())
    assert set(ref["contact_blocks"]) <= seen          # every active coupling is in the pattern
    assert err <= tol * scale


MODES = ["compact", "branch"]


def _mode(symx, name):
    return symx.SYMX_CONTACT_BRANCH if name == "branch" else symx.SYMX_CONTACT_COMPACT


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_contact_assembly(symx, precision, mode):
    """Both activation modes: compaction of the active candidates, and the
    activation as a branch of the generated element function (every candidate
    evaluated, inactive ones through the zero arm)."""
    scene = sg.contact_stack_scene(4)
    mesh = symx.Mesh(scene)
    cl = scene.contacts
    mesh.set_contact_mode(_mode(symx, mode))
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    E, g, vals = mesh.assemble(scene.x0, xt, dt, FLAGS, p)
    ref = assembly.assemble(scene, scene.x0, xt, dt)
    act = contact.activation(scene.x0[cl.tuples], cl.dhat) > 0
    assert 0 < act.sum() < act.size                      # some active, some not
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < tol
    assert rel(_bsr(vals), ref["vals"]) < tol
    _check_contact_blocks(mesh, ref, p, tol)
    mesh.close()


@pytest.mark.parametrize("mode", MODES)
def test_contact_compaction_many_candidates(symx, mode):
    """3,528 candidates (two compaction chunks), activity by distance."""
    scene = sg.contact_stack_scene(6, seed=10)
    tuples = _all_triangles(scene, 6)
    scene.contacts = sg.ContactList(tuples, kc=1e3, dhat=1e-3)
    mesh = symx.Mesh(scene)
    mesh.set_contact_mode(_mode(symx, mode))
    mesh.set_contacts(tuples, 1e3, 1e-3)
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    E, g, vals = mesh.assemble(scene.x0, xt, scene.dt, FLAGS, symx.SYMX_F64)
    ref = assembly.assemble(scene, scene.x0, xt, scene.dt)
    assert abs(E - ref["E"]) <= F64_TOL * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < F64_TOL
    _check_contact_blocks(mesh, ref, symx.SYMX_F64, F64_TOL)
    mesh.close()


@pytest.mark.parametrize("mode", MODES)
def test_contact_projected(symx, mode):
    scene = sg.contact_stack_scene(4, seed=11)
    cl = scene.contacts
    mesh = symx.Mesh(scene)
    mesh.set_contact_mode(_mode(symx, mode))
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    ref = assembly.assemble(scene, scene.x0, xt, scene.dt, project=True)
    raw = assembly.assemble(scene, scene.x0, xt, scene.dt)
    d = max(np.abs(ref["contact_blocks"][k] - raw["contact_blocks"][k]).max()
            for k in ref["contact_blocks"])
    assert d > 0                                          # the projection acts on contacts
    for p, tol in ((symx.SYMX_F64, F64_TOL), (symx.SYMX_F32, F32_TOL)):
        E, g, vals = mesh.assemble(scene.x0, xt, scene.dt, FLAGS | symx.SYMX_PROJECT_PSD, p)
        assert rel(_bsr(vals), ref["vals"]) < tol
        _check_contact_blocks(mesh, ref, p, tol)
    mesh.close()


def test_contact_list_changes(symx):
    """Dynamic topology: the couplings follow the candidate list."""
    scene = sg.contact_stack_scene(4, seed=12)
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    full = scene.contacts.tuples
    # sizes: n, n/3 (buffers reused), a longer list (buffers grown), empty
    # (buffers freed), one candidate repeated (two contributions per block), n
    rep = np.repeat(full[:1], 2, axis=0)
    for tuples in (full, full[::3], _all_triangles(scene, 4)[5::7], full[:0], rep, full):
        scene.contacts = sg.ContactList(tuples, kc=1e3, dhat=1e-3) if len(tuples) else None
        mesh.set_contacts(tuples, 1e3, 1e-3)
        E, g, vals = mesh.assemble(scene.x0, xt, scene.dt, FLAGS, symx.SYMX_F64)
        ref = assembly.assemble(scene, scene.x0, xt, scene.dt)
        assert abs(E - ref["E"]) <= F64_TOL * abs(ref["E"])
        assert rel(g.cpu().numpy(), ref["g"]) < F64_TOL
        assert rel(_bsr(vals), ref["vals"]) < F64_TOL
        if len(tuples):
            _check_contact_blocks(mesh, ref, symx.SYMX_F64, F64_TOL)
            rp, ci, _ = mesh.contact_bsr(symx.SYMX_F64)
            rp_o, ci_o = _expected_pattern(tuples, scene.n_nodes)
            assert np.array_equal(rp, rp_o) and np.array_equal(ci, ci_o)   # bit-exact pattern
        else:
            assert mesh.contact_bsr()[1].size == 0
    mesh.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_contact_newton_step(symx, precision, mode):
    """The upper cube moves down onto the barrier: one implicit-Euler step
    reaches the oracle's minimiser, every active point stays above its plane."""
    scene = sg.contact_stack_scene(4, seed=13)
    cl = scene.contacts
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    mesh = symx.Mesh(scene)
    mesh.set_contact_mode(_mode(symx, mode))
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
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
    d, _, _ = contact.point_plane_distance(xh[cl.tuples])
    assert d.min() > 0


def test_contact_penetration_and_invalid(symx):
    scene = sg.contact_stack_scene(3, seed=14)
    mesh = symx.Mesh(scene)
    cl = scene.contacts
    x = scene.x0.copy()
    x[cl.tuples[0, 0], 2] -= 5e-3                          # through the plane
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
    with pytest.raises(symx.SymxError, match="NONFINITE"):
        mesh.assemble(x, None, 0.0, 1, symx.SYMX_F64)
    bad = cl.tuples.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contacts(bad, cl.kc, cl.dhat)
    bad = cl.tuples.copy()
    bad[0, 2] = scene.n_nodes
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contacts(bad, cl.kc, cl.dhat)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contacts(cl.tuples, -1.0, cl.dhat)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        mesh.set_contact_mode(2)
    # the branch mode reports the penetration as the compaction mode does
    mesh.set_contact_mode(symx.SYMX_CONTACT_BRANCH)
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
    with pytest.raises(symx.SymxError, match="NONFINITE"):
        mesh.assemble(x, None, 0.0, 1, symx.SYMX_F64)
    mesh.close()
