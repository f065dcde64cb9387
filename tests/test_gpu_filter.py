"""Stable Neo-Hookean tets with the density Hessian filtered to PSD through its
analytic eigensystem (SYMX_PROJECT_FILTER, Newton project = 2), on the HIP
path through the C-ABI, against the float64 oracle (which clamps the
eigenvalues of the 9x9 density Hessian numerically).  Other element kinds
take the nearest-PSD projection in this mode.

Tolerances: normwise 1e-10 in float64, 1e-4 in float32.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements, newton, rest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL = 1e-4


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


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_filtered_elem_hessians(symx, precision):
    """Stressed single tets (20% inverted, 30% compressed), per element."""
    n = 3000
    x, X = sg.random_tets(n, 91)
    conn = np.arange(4 * n, dtype=np.int32).reshape(n, 4)
    young = np.exp(np.random.default_rng(92).uniform(np.log(1e4), np.log(1e7), n))
    es = sg.EnergySet(sg.SNH_TET4, conn, young_per_elem=young, poisson=0.4)
    Xf, xf = X.reshape(-1, 3), x.reshape(-1, 3)
    scene = sg.Scene("loose", Xf, [es], np.zeros(Xf.shape[0], np.uint8), xf, np.zeros_like(Xf))
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
             | symx.SYMX_PROJECT_FILTER)
    E, g, H = mesh.eval_derivatives(0, xf, flags=flags, precision=p)
    mu, lam = rest.lame(young, 0.4)
    Eo, go, Ho = elements.snh_tet4_filtered(x, X, mu, lam)
    assert rel(E.cpu().numpy(), Eo) < tol
    assert rel(g.cpu().numpy().reshape(n, 4, 3), go) < tol
    Hd = H.cpu().numpy().reshape(n, 12, 12)
    Hr = Ho.reshape(n, 12, 12)
    assert max(rel(Hd[e], Hr[e]) for e in range(0, n, 3)) < tol
    _, _, Hraw = elements.snh_tet4(x, X, mu, lam)
    assert rel(Hraw.reshape(n, 12, 12), Hr) > 1e-3          # the filter is not a no-op
    mesh.close()


def test_filtered_assembly_c1(symx):
    scene = sg.config_c1()
    x = scene.x0 + np.random.default_rng(93).uniform(-2e-3, 2e-3, size=scene.x0.shape)
    x[scene.fixed.astype(bool)] = scene.X[scene.fixed.astype(bool)]
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
             | symx.SYMX_PROJECT_FILTER)
    ref = assembly.assemble(scene, x, xt, 0.01, project="filter")
    raw = assembly.assemble(scene, x, xt, 0.01, project=False)
    psd = assembly.assemble(scene, x, xt, 0.01, project=True)
    assert rel(raw["vals"], ref["vals"]) > 1e-6
    assert rel(psd["vals"], ref["vals"]) > 1e-6                # a different projection
    for p, tol in ((symx.SYMX_F64, F64_TOL), (symx.SYMX_F32, F32_TOL)):
        E, g, vals = mesh.assemble(x, xt, 0.01, flags, p)
        assert rel(_bsr(vals), ref["vals"]) < tol
        assert rel(g.cpu().numpy(), ref["g"]) < tol
        assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    mesh.close()


def test_filtered_assembly_mixed_kinds(symx):
    """SNH tets filtered, cloth membranes projected, hinges as they are."""
    s = sg.tet_cube_scene(3, seed=7, perturb=0.05)
    c = sg.cloth_scene(5, perturb=0.2)
    N = s.n_nodes
    es = [s.energies[0]] + [sg.EnergySet(e.kind, e.conn + N, young=e.young, poisson=e.poisson,
                                         thickness=e.thickness, bend_kb=e.bend_kb,
                                         density=e.density) for e in c.energies]
    X = np.concatenate([s.X, c.X])
    scene = sg.Scene("mixed", X, es, np.concatenate([s.fixed, c.fixed]),
                     np.concatenate([s.x0, c.x0]), np.zeros_like(X), dt=0.01)
    x = scene.x0 + np.random.default_rng(94).normal(scale=0.02, size=scene.x0.shape)
    x[scene.fixed.astype(bool)] = scene.X[scene.fixed.astype(bool)]
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = (symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
             | symx.SYMX_PROJECT_FILTER)
    ref = assembly.assemble(scene, x, xt, 0.01, project="filter")
    for p, tol in ((symx.SYMX_F64, F64_TOL), (symx.SYMX_F32, F32_TOL)):
        _, g, vals = mesh.assemble(x, xt, 0.01, flags, p)
        assert rel(_bsr(vals), ref["vals"]) < tol
        assert rel(g.cpu().numpy(), ref["g"]) < tol
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_newton_step_filtered_c1(symx, precision):
    scene = sg.config_c1()
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=scene.dt, precision=p, project=2))
    mesh.close()
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xh = x.cpu().numpy()
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, dt, want_hess=False)["g"])
    g = assembly.assemble(scene, xh, xt, dt, want_hess=False)["g"]
    assert np.linalg.norm(g) <= 1.01e-6 * r0
    ok, xo, repo = newton.newton_solve(scene, scene.x0, scene.v0, dt,
                                       newton.StepParams(dt=dt, project="filter"))
    assert ok
    m_min = rest.lumped_mass(scene).min()
    assert np.max(np.abs(xh - xo)) <= 2.0e-6 * r0 * dt * dt / m_min
    assert rep.energy == pytest.approx(repo["energy"], rel=1e-9)


def test_invalid_projection_mode_rejected(symx):
    scene = sg.config_c1()
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(x)
    st, _ = mesh.newton_step(x, v, symx.step_params(dt=scene.dt, project=3))
    mesh.close()
    assert symx.STATUS[st] == "INVALID_ARG"
