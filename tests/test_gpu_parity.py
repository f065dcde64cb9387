"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances (normwise, max|a-b| / max|b| per output array): 1e-10 in float64,
1e-4 in float32 (the element kernels, Hessian values and PCG in single
precision).  Integer outputs (pattern, scatter map) are compared bit for bit.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements, newton, projection, rest

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


def loose_tet_scene(n_elem, seed):
    """Disjoint stressed tets (inverted / compressed / stretched): one scene."""
    x, X = sg.random_tets(n_elem, seed)
    conn = np.arange(4 * n_elem, dtype=np.int32).reshape(n_elem, 4)
    es = sg.EnergySet(sg.SNH_TET4, conn, young_per_elem=np.exp(
        np.random.default_rng(seed).uniform(np.log(1e4), np.log(1e7), n_elem)), poisson=0.4)
    Xf = X.reshape(-1, 3)
    return sg.Scene("loose", Xf, [es], np.zeros(Xf.shape[0], np.uint8), x.reshape(-1, 3),
                    np.zeros_like(Xf)), x.reshape(-1, 3)


def mixed_scene():
    """Tet block + cloth (membrane + hinges) in one global system, perturbed."""
    s = sg.tet_cube_scene(3, seed=7, perturb=0.05)
    c = sg.cloth_scene(5, perturb=0.2)
    N = s.n_nodes
    es = [s.energies[0]] + [sg.EnergySet(e.kind, e.conn + N, young=e.young, poisson=e.poisson,
                                         thickness=e.thickness, bend_kb=e.bend_kb,
                                         density=e.density) for e in c.energies]
    X = np.concatenate([s.X, c.X])
    return sg.Scene("mixed", X, es, np.concatenate([s.fixed, c.fixed]),
                    np.concatenate([s.x0, c.x0]), np.zeros_like(X), dt=0.01)


# ---------------------------------------------------------------------------
# pattern, scatter map, masses
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["c1", "mixed"])
def test_pattern_and_scatter_map_bit_exact(symx, which):
    scene = sg.config_c1() if which == "c1" else mixed_scene()
    mesh = symx.Mesh(scene)
    rp, ci, maps = mesh.pattern()
    rp_o, ci_o = assembly.pattern_fast(scene)
    assert np.array_equal(rp, rp_o)
    assert np.array_equal(ci, ci_o)
    for es, m in zip(scene.energies, maps):
        assert np.array_equal(m, assembly._block_index(es.conn, rp_o, ci_o))
    assert mesh.info.nnzb == ci_o.size
    assert rel(mesh.masses(), rest.lumped_mass(scene)) < 1e-14
    mesh.close()


# ---------------------------------------------------------------------------
# per-element derivatives
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_elem_derivatives_stressed_tets(symx, precision):
    scene, x = loose_tet_scene(3000, 5)
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    E, g, H = mesh.eval_derivatives(0, x, precision=p)
    Eo, go, Ho = elements.element_eval(scene.energies[0], x, scene.X)
    tol = F64_TOL if precision == "f64" else F32_TOL
    n = Eo.shape[0]
    # energies: per element (SNH has a large rest offset, so compare per element)
    assert rel(E.cpu().numpy(), Eo) < tol
    assert rel(g.cpu().numpy().reshape(n, 4, 3), go) < tol
    Hd = H.cpu().numpy().reshape(n, 12, 12)
    Hr = Ho.reshape(n, 12, 12)
    worst = max(rel(Hd[e], Hr[e]) for e in range(0, n, 7))
    assert worst < tol
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_elem_derivatives_cloth(symx, precision):
    scene = sg.cloth_scene(6, perturb=0.3)
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    x = scene.x0 + np.random.default_rng(2).normal(scale=0.01, size=scene.x0.shape)
    for si, es in enumerate(scene.energies):
        E, g, H = mesh.eval_derivatives(si, x, precision=p)
        Eo, go, Ho = elements.element_eval(es, x, scene.X)
        k = es.conn.shape[1]
        n = es.conn.shape[0]
        assert rel(E.cpu().numpy(), Eo) < tol, si
        assert rel(g.cpu().numpy().reshape(n, k, 3), go) < tol, si
        assert rel(H.cpu().numpy().reshape(n, 3 * k, 3 * k), Ho.reshape(n, 3 * k, 3 * k)) < tol, si
    mesh.close()


def test_elem_projection_matches_eigh(symx):
    scene, x = loose_tet_scene(600, 9)
    mesh = symx.Mesh(scene)
    flags = symx.SYMX_EVAL_HESS | symx.SYMX_PROJECT_PSD
    _, _, H = mesh.eval_derivatives(0, x, flags=flags, precision=symx.SYMX_F64)
    _, _, Ho = elements.element_eval(scene.energies[0], x, scene.X)
    Po = projection.project_psd(Ho.reshape(-1, 12, 12))
    Hd = H.cpu().numpy()
    n_neg = np.sum(np.linalg.eigvalsh(Ho.reshape(-1, 12, 12)).min(axis=1) < 0)
    assert n_neg > 50  # the stressed set really exercises the projection
    for e in range(Hd.shape[0]):
        assert rel(Hd[e], Po[e]) < F64_TOL, e
    _, _, H32 = mesh.eval_derivatives(0, x, flags=flags, precision=symx.SYMX_F32)
    H32 = H32.cpu().numpy()
    worst = max(rel(H32[e], Po[e]) for e in range(H32.shape[0]))
    assert worst < F32_TOL
    mesh.close()


def test_elem_projection_membrane_and_hinge_match_eigh(symx):
    """9x9 membrane and 12x12 hinge Hessians of a strongly perturbed cloth: the
    projection of each element equals the eigendecomposition-based oracle.
    Errors are measured against the element's unprojected Hessian: the nearest
    PSD map is 1-Lipschitz, and a fully compressed membrane projects to zero,
    where an error relative to the result itself has no scale."""
    scene = sg.cloth_scene(6, perturb=0.3)
    x = scene.x0 + np.random.default_rng(12).normal(scale=0.03, size=scene.x0.shape)
    mesh = symx.Mesh(scene)
    flags = symx.SYMX_EVAL_HESS | symx.SYMX_PROJECT_PSD
    for si, es in enumerate(scene.energies):
        D = 3 * es.conn.shape[1]
        _, _, Ho = elements.element_eval(es, x, scene.X)
        Ho = Ho.reshape(-1, D, D)
        Po = projection.project_psd(Ho)
        for p, tol in ((symx.SYMX_F64, F64_TOL), (symx.SYMX_F32, F32_TOL)):
            _, _, H = mesh.eval_derivatives(si, x, flags=flags, precision=p)
            Hd = H.cpu().numpy().astype(np.float64).reshape(-1, D, D)
            worst = max(np.max(np.abs(Hd[e] - Po[e])) / np.max(np.abs(Ho[e]))
                        for e in range(Hd.shape[0]))
            assert worst < tol, (si, p, worst)
    n_neg = np.sum(np.linalg.eigvalsh(
        elements.element_eval(scene.energies[0], x, scene.X)[2].reshape(-1, 9, 9)).min(axis=1)
        < -1e-9)
    assert n_neg > 10  # the membrane set really exercises the projection
    mesh.close()


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------
def _bsr(vals):
    return vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3)


@pytest.mark.parametrize("which", ["c1", "mixed"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_assembly_matches_oracle(symx, which, precision):
    scene = sg.config_c1() if which == "c1" else mixed_scene()
    mesh = symx.Mesh(scene)
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.x0 * 0 + 0.05, dt, scene.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    E, g, vals = mesh.assemble(scene.x0, xt, dt, flags, p)
    ref = assembly.assemble(scene, scene.x0, xt, dt)
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < tol
    assert rel(_bsr(vals), ref["vals"]) < tol
    # elastic only, no Dirichlet
    flags2 = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
    E2, g2, v2 = mesh.assemble(scene.x0, None, 0.0, flags2, p)
    ref2 = assembly.assemble(scene, scene.x0, dirichlet=False)
    assert abs(E2 - ref2["E"]) <= tol * abs(ref2["E"])
    assert rel(g2.cpu().numpy(), ref2["g"]) < tol
    assert rel(_bsr(v2), ref2["vals"]) < tol
    mesh.close()


def test_projected_assembly_c1(symx):
    scene = sg.config_c1()
    x = scene.x0 + np.random.default_rng(4).uniform(-2e-3, 2e-3, size=scene.x0.shape)
    x[scene.fixed.astype(bool)] = scene.X[scene.fixed.astype(bool)]
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
             | symx.SYMX_PROJECT_PSD)
    E, g, vals = mesh.assemble(x, xt, 0.01, flags, symx.SYMX_F64)
    ref = assembly.assemble(scene, x, xt, 0.01, project=True)
    raw = assembly.assemble(scene, x, xt, 0.01, project=False)
    assert rel(raw["vals"], ref["vals"]) > 1e-6  # projection is not a no-op here
    assert rel(_bsr(vals), ref["vals"]) < F64_TOL
    assert rel(g.cpu().numpy(), ref["g"]) < F64_TOL
    E32, g32, v32 = mesh.assemble(x, xt, 0.01, flags, symx.SYMX_F32)
    assert rel(_bsr(v32), ref["vals"]) < F32_TOL
    mesh.close()


def test_projected_assembly_mixed(symx):
    scene = mixed_scene()
    x = scene.x0 + np.random.default_rng(5).normal(scale=0.02, size=scene.x0.shape)
    x[scene.fixed.astype(bool)] = scene.X[scene.fixed.astype(bool)]
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
             | symx.SYMX_PROJECT_PSD)
    ref = assembly.assemble(scene, x, xt, 0.01, project=True)
    raw = assembly.assemble(scene, x, xt, 0.01, project=False)
    assert rel(raw["vals"], ref["vals"]) > 1e-6
    for p, tol in ((symx.SYMX_F64, F64_TOL), (symx.SYMX_F32, F32_TOL)):
        E, g, vals = mesh.assemble(x, xt, 0.01, flags, p)
        assert rel(_bsr(vals), ref["vals"]) < tol
        assert rel(g.cpu().numpy(), ref["g"]) < tol
    mesh.close()


def test_assembly_bitwise_reproducible(symx):
    scene = mixed_scene()
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    for p in (symx.SYMX_F64, symx.SYMX_F32):
        outs = [mesh.assemble(scene.x0, xt, 0.01, flags, p) for _ in range(3)]
        for E, g, v in outs[1:]:
            assert E == outs[0][0]
            assert torch.equal(g, outs[0][1])
            assert torch.equal(v, outs[0][2])
    mesh.close()


@pytest.mark.parametrize("mode", ["psd", "filter"])
def test_projected_assembly_bitwise_reproducible(symx, mode):
    """Projected (records path) and filtered assembly at a strained state give
    the same bits on every call: fixed reduction orders, no atomics."""
    scene = sg.tet_cube_scene(5, seed=41, perturb=0.2)
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    proj = symx.SYMX_PROJECT_PSD if mode == "psd" else symx.SYMX_PROJECT_FILTER
    flags = (symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
             | proj)
    for p in (symx.SYMX_F64, symx.SYMX_F32):
        outs = [mesh.assemble(scene.x0, xt, 0.01, flags, p) for _ in range(3)]
        for E, g, v in outs[1:]:
            assert E == outs[0][0]
            assert torch.equal(g, outs[0][1])
            assert torch.equal(v, outs[0][2])
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_newton_step_bitwise_reproducible(symx, precision):
    """The same implicit-Euler step from the same state, twice: identical
    positions, velocities and iteration counts."""
    scene = sg.tet_cube_scene(6, seed=42, perturb=0.1, vel_std=0.1)
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    runs = []
    for _ in range(2):
        x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
        v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01, precision=p))
        assert st == 0
        runs.append((x, v, rep.as_dict()))
    (xa, va, ra), (xb, vb, rb) = runs
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert ra["newton_iters"] == rb["newton_iters"] and ra["pcg_iters"] == rb["pcg_iters"]
    assert ra["energy"] == rb["energy"]
    mesh.close()


def test_bsr_symmetry_and_matvec(symx):
    scene = sg.config_c1()
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, 0.01, scene.gravity)
    flags = symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
    _, _, vals = mesh.assemble(scene.x0, xt, 0.01, flags, symx.SYMX_F64)
    rp, ci, _ = mesh.pattern()
    A = assembly.to_scipy(rp, ci, _bsr(vals))
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    p = np.random.default_rng(1).normal(size=3 * scene.n_nodes)
    y = A @ p
    ref = rest.lumped_mass(scene).repeat(3) / 1e-4 * p
    _, _, He = elements.element_eval(scene.energies[0], scene.x0, scene.X)
    c = scene.energies[0].conn
    ye = np.einsum("emn,en->em", He.reshape(-1, 12, 12), p.reshape(-1, 3)[c].reshape(-1, 12))
    refv = ref.reshape(-1, 3)
    np.add.at(refv, c.ravel(), ye.reshape(-1, 3))
    assert rel(y, refv.ravel()) < F64_TOL
    mesh.close()


# ---------------------------------------------------------------------------
# Newton step
# ---------------------------------------------------------------------------
def _newton(symx, scene, precision, **kw):
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    prm = symx.step_params(dt=scene.dt, precision=precision, **kw)
    st, rep = mesh.newton_step(x, v, prm)
    mesh.close()
    return st, rep, x.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_newton_step_c1(symx, precision):
    scene = sg.config_c1()
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    st, rep, x, v = _newton(symx, scene, p)
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    # the oracle's float64 gradient at the device's answer meets the tolerance
    g = assembly.assemble(scene, x, xt, dt, want_hess=False)["g"]
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, dt, want_hess=False)["g"])
    assert rep.residual0 == pytest.approx(r0, rel=1e-10)
    assert np.linalg.norm(g) <= 1.01e-6 * r0
    assert np.allclose(v, (x - scene.x0) / dt)
    # same minimiser as the oracle's own Newton step (agreement within the
    # solver tolerance: |dx| <= |H^-1| |g| with |H^-1| <= dt^2 / m_min)
    ok, xo, repo = newton.newton_solve(scene, scene.x0, scene.v0, dt, newton.StepParams(dt=dt))
    assert ok
    m_min = rest.lumped_mass(scene).min()
    bound = 2.0e-6 * r0 * dt * dt / m_min
    assert np.max(np.abs(x - xo)) <= bound
    assert rep.energy == pytest.approx(repo["energy"], rel=1e-9)


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_newton_step_projected_c1(symx, precision):
    """Newton with per-element PSD projection (the fused evaluation +
    projection path) converges and reaches the oracle's projected step."""
    scene = sg.config_c1()
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    st, rep, x, v = _newton(symx, scene, p, project=1)
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, dt, want_hess=False)["g"])
    g = assembly.assemble(scene, x, xt, dt, want_hess=False)["g"]
    assert np.linalg.norm(g) <= 1.01e-6 * r0
    ok, xo, repo = newton.newton_solve(scene, scene.x0, scene.v0, dt,
                                       newton.StepParams(dt=dt, project=True))
    assert ok
    m_min = rest.lumped_mass(scene).min()
    assert np.max(np.abs(x - xo)) <= 2.0e-6 * r0 * dt * dt / m_min
    assert rep.energy == pytest.approx(repo["energy"], rel=1e-9)


def test_f32_refinement_reaches_float64_accuracy(symx):
    """Mixed-precision iterative refinement (F32_REFINED).  With the forcing
    term capped at 1e-9, far below what a float32 PCG on the rounded Hessian
    reaches (about 1e-6 relative to the float64 Hessian), each linear solve is
    refined until |b - H dx| <= 1e-9 |b| with H the float64 Hessian; with no
    refinement passes the same solves stop at the float32 floor."""
    scene = sg.config_c1()
    out = {}
    for mr in (0, 4):
        st, rep, x, _ = _newton(symx, scene, symx.SYMX_F32_REFINED, forcing_max=1e-9,
                                max_refine=mr)
        assert st == 0, (symx.STATUS[st], rep.as_dict())
        out[mr] = (rep, x)
    rep0, _ = out[0]
    rep4, x4 = out[4]
    assert rep0.refinements == 0 and rep0.lin_residual > 1e-8, rep0.as_dict()
    assert rep4.refinements >= rep4.newton_iters >= 1, rep4.as_dict()
    assert 0.0 <= rep4.lin_residual <= 1e-9, rep4.as_dict()
    # the refined solves behave as exact ones: the oracle's Newton step with
    # direct sparse solves reaches the same minimiser in as many iterations
    dt = scene.dt
    ok, xo, repo = newton.newton_solve(scene, scene.x0, scene.v0, dt, newton.StepParams(dt=dt),
                                       solver="direct")
    assert ok
    assert abs(rep4.newton_iters - repo["newton_iters"]) <= 1
    m_min = rest.lumped_mass(scene).min()
    assert np.max(np.abs(x4 - xo)) <= 2.0e-6 * rep4.residual0 * dt * dt / m_min
    # float64 mode reports no refinement residual
    st, rep64, _, _ = _newton(symx, scene, symx.SYMX_F64)
    assert st == 0 and rep64.lin_residual == -1.0 and rep64.refinements == 0
    # forcing terms outside (0, 1) and negative pass counts are rejected
    for kw in (dict(forcing_max=0.0), dict(forcing_max=1.0), dict(max_refine=-1)):
        st, _, _, _ = _newton(symx, scene, symx.SYMX_F32_REFINED, **kw)
        assert symx.STATUS[st] == "INVALID_ARG", kw


def test_newton_step_mixed_f32_refined(symx):
    scene = mixed_scene()
    st, rep, x, _ = _newton(symx, scene, symx.SYMX_F32_REFINED)
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    g = assembly.assemble(scene, x, xt, scene.dt, want_hess=False)["g"]
    assert np.linalg.norm(g) <= 1.01e-6 * rep.residual0


def test_newton_rigid_translation_exact(symx):
    s = sg.tet_cube_scene(3, seed=2, perturb=0.0)
    s.fixed[:] = 0
    s.v0 = np.tile(np.array([[0.3, -0.1, 0.2]]), (s.n_nodes, 1))
    st, rep, x, v = _newton(symx, s, symx.SYMX_F64, gravity=(0.0, 0.0, 0.0))
    assert st == 0
    # exact answer X + dt v; Newton stops at |g| <= 1e-6 r0 and H >= M/dt^2 at
    # rest, so the error is at most dt^2/m_min * 1e-6 r0
    bound = s.dt ** 2 / rest.lumped_mass(s).min() * 1.01e-6 * rep.residual0
    assert np.max(np.abs(x - (s.X + s.dt * s.v0))) <= bound


@pytest.mark.parametrize("precision", ["f64", "f32r"])
def test_newton_free_fall_closed_form(symx, precision):
    """A free body under gravity (Eq. 2-3): every implicit-Euler step moves all
    nodes as one particle, v_{k+1} = v_k + dt g, x_{k+1} = x_k + dt v_{k+1};
    after K steps x_K = x_0 + K dt v_0 + dt^2 g K (K + 1) / 2 (a closed form,
    not the oracle)."""
    s = sg.tet_cube_scene(3, seed=2, perturb=0.0)
    s.fixed[:] = 0
    grav = np.array([0.7, -0.4, -9.81])
    v0 = np.array([0.05, 0.02, -0.1])
    dt, K = 0.01, 5
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32_REFINED
    mesh = symx.Mesh(s)
    x = torch.tensor(s.X, dtype=torch.float64, device="cuda")
    v = torch.tensor(np.tile(v0, (s.n_nodes, 1)), dtype=torch.float64, device="cuda")
    bound = 0.0
    m_min = rest.lumped_mass(s).min()
    for _ in range(K):
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, precision=p,
                                                          gravity=tuple(grav)))
        assert st == 0 and rep.dt_halvings == 0, (symx.STATUS[st], rep.as_dict())
        # Newton stops at |g| <= 1e-6 r0 and H >= M / dt^2 for a translation
        bound += dt * dt / m_min * 1.01e-6 * rep.residual0
    x_ref = s.X + K * dt * v0 + dt * dt * grav * K * (K + 1) / 2
    assert np.max(np.abs(x.cpu().numpy() - x_ref)) <= bound + 1e-13
    assert np.max(np.abs(v.cpu().numpy() - (v0 + K * dt * grav))) <= bound / dt * 2 + 1e-11
    mesh.close()


def test_nonfinite_input_is_reported(symx):
    scene = sg.tet_cube_scene(2, seed=1)
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    x[3, 1] = float("nan")
    v = torch.zeros_like(x)
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01))
    assert symx.STATUS[st] == "NONFINITE"
    # the mesh stays usable afterwards
    x[3, 1] = float(scene.x0[3, 1])
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01))
    assert st == 0
    mesh.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_assembly_reports_nonfinite_and_recovers(symx, precision):
    """A NaN position makes the assembly call report NONFINITE (the energy and
    the flag come back together); the flag is cleared, so the next call with
    finite positions succeeds and matches the oracle's energy."""
    scene = sg.tet_cube_scene(2, seed=3, perturb=0.05)
    mesh = symx.Mesh(scene)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
    x = scene.x0.copy()
    x[5, 0] = np.nan
    with pytest.raises(symx.SymxError, match="NONFINITE"):
        mesh.assemble(x, None, 0.0, flags, p)
    E, g, _ = mesh.assemble(scene.x0, None, 0.0, flags, p)
    ref = assembly.assemble(scene, scene.x0, None, 0.0, want_hess=False)
    tol = 1e-10 if precision == "f64" else 1e-4
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    assert np.all(np.isfinite(g.cpu().numpy()))
    mesh.close()


def test_forced_failures_halve_dt(symx):
    scene = sg.tet_cube_scene(2, seed=1)
    st, rep, x, _ = _newton(symx, scene, symx.SYMX_F64, max_newton=0, max_halvings=3)
    assert symx.STATUS[st] == "NOT_CONVERGED"
    assert rep.dt_halvings == 3 and rep.dt_used == pytest.approx(0.01 / 8)
    assert np.array_equal(x, scene.x0)  # unchanged on failure


def test_uncontrolled_step_takes_the_given_dt(symx):
    """After a step that succeeded only at a halved dt, the mesh keeps the
    reduced dt for its next controlled step; a step with max_halvings = 0 is
    taken at exactly the given dt and leaves that state alone."""
    scene = sg.config_c4(6)
    # the smallest Newton iteration limit with which the first step succeeds
    # (smaller steps need fewer iterations, so it succeeds after halvings)
    reduced = None
    for max_newton in range(2, 40):
        mesh = symx.Mesh(scene)
        x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
        v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01, max_newton=max_newton,
                                                          max_halvings=6))
        if st == 0:
            reduced = rep.dt_used if rep.dt_halvings > 0 else None
            break
        mesh.close()
    assert reduced is not None and reduced < 0.01
    x1, v1 = x.clone(), v.clone()
    st, rep = mesh.newton_step(x1, v1, symx.step_params(dt=0.01, max_halvings=0))
    assert st == 0 and rep.dt_used == 0.01 and rep.dt_halvings == 0
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01, max_newton=100, max_halvings=6))
    assert st == 0 and rep.dt_used == reduced
    mesh.close()


def test_invalid_mesh_rejected(symx):
    s = sg.tet_cube_scene(1, seed=1)
    s.energies[0].conn = s.energies[0].conn.copy()
    s.energies[0].conn[0, 0] = 999
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        symx.Mesh(s)


def _edge_scene():
    """Tet block, an empty membrane set and three isolated nodes (rows with
    only a diagonal block), one fixed isolated node."""
    s = sg.tet_cube_scene(3, seed=7, perturb=0.05)
    iso = np.array([[1.0, 1.0, 1.0], [1.1, 1.0, 1.0], [1.0, 1.2, 1.0]])
    X = np.concatenate([s.X, iso])
    x0 = np.concatenate([s.x0, iso + 0.001])
    es = [s.energies[0], sg.EnergySet(sg.STVK_TRI3, np.zeros((0, 3), np.int32), young=1e4,
                                      poisson=0.3, thickness=1e-3)]
    fixed = np.concatenate([s.fixed, np.array([0, 0, 1], np.uint8)])
    return sg.Scene("edge", X, es, fixed, x0, np.zeros_like(X), dt=0.01)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_empty_set_and_isolated_nodes(symx, precision):
    scene = _edge_scene()
    mesh = symx.Mesh(scene)
    rp, ci, _ = mesh.pattern()
    rp_o, ci_o = assembly.pattern_fast(scene)
    assert np.array_equal(rp, rp_o) and np.array_equal(ci, ci_o)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    for extra in (0, symx.SYMX_PROJECT_PSD):
        E, g, vals = mesh.assemble(scene.x0, xt, scene.dt, flags | extra, p)
        ref = assembly.assemble(scene, scene.x0, xt, scene.dt, project=bool(extra))
        assert abs(E - ref["E"]) <= tol * abs(ref["E"])
        assert rel(g.cpu().numpy(), ref["g"]) < tol
        assert rel(_bsr(vals), ref["vals"]) < tol
    E1, g1, H1 = mesh.eval_derivatives(1, scene.x0, precision=p)  # the empty set
    assert E1.numel() == 0
    st, rep, x, v = _newton(symx, scene, p if p == symx.SYMX_F64 else symx.SYMX_F32_REFINED)
    assert st == 0
    mesh.close()


def test_single_element(symx):
    x, X = sg.random_tets(1, seed=3)
    conn = np.arange(4, dtype=np.int32).reshape(1, 4)
    es = sg.EnergySet(sg.SNH_TET4, conn, young=1e5, poisson=0.4)
    scene = sg.Scene("one", X.reshape(4, 3), [es], np.zeros(4, np.uint8), x.reshape(4, 3),
                     np.zeros((4, 3)))
    mesh = symx.Mesh(scene)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS
    E, g, vals = mesh.assemble(scene.x0, None, 0.0, flags, symx.SYMX_F64)
    ref = assembly.assemble(scene, scene.x0, dirichlet=False)
    assert abs(E - ref["E"]) <= F64_TOL * abs(ref["E"])
    assert rel(g.cpu().numpy(), ref["g"]) < F64_TOL
    assert rel(_bsr(vals), ref["vals"]) < F64_TOL
    mesh.close()


def test_invalid_elements_rejected(symx):
    """Degenerate rest tet, repeated node, a node in more than 256 elements."""
    s = sg.tet_cube_scene(1, seed=1)
    flat = s.energies[0].conn.copy()
    X = s.X.copy()
    X[flat[0]] = X[flat[0, 0]] + np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]]) * 1e-3
    bad = sg.Scene("degenerate", X, [s.energies[0]], s.fixed, X.copy(), np.zeros_like(X))
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        symx.Mesh(bad)
    rep = s.energies[0].conn.copy()
    rep[0, 1] = rep[0, 0]
    s2 = sg.Scene("repeat", s.X, [sg.EnergySet(sg.SNH_TET4, rep)], s.fixed, s.x0, s.v0)
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        symx.Mesh(s2)
    # 257 tets sharing node 0 (a fan of thin tets around the z axis)
    n = 257
    ang = 2 * np.pi * np.arange(n + 1) / n
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(n + 1)], axis=1) * 0.01
    Xf = np.concatenate([np.zeros((1, 3)), np.array([[0, 0, 0.01]]), ring[:n]])
    conn = np.array([[0, 2 + i, 2 + (i + 1) % n, 1] for i in range(n)], np.int32)
    fan = sg.Scene("fan", Xf, [sg.EnergySet(sg.SNH_TET4, conn)], np.zeros(len(Xf), np.uint8),
                   Xf.copy(), np.zeros_like(Xf))
    with pytest.raises(symx.SymxError, match="INVALID_ARG"):
        symx.Mesh(fan)


def test_f32_refined_tracks_f64_trajectory(symx):
    """Stiff heterogeneous compressed block (the C4 recipe at n=6): the FP32-
    refined steps, taken with the FP64 run's time steps, stay within the Newton
    tolerance of the FP64 trajectory."""
    scene = sg.config_c4(6)
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    dts, E64 = [], []
    for _ in range(4):
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=0.01, precision=symx.SYMX_F64))
        assert st == 0
        dts.append(rep.dt_used)
        E64.append(rep.energy)
    x64 = x.cpu().numpy()
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    for dt in dts:
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, precision=symx.SYMX_F32_REFINED,
                                                          max_halvings=0))
        assert st == 0 and rep.dt_used == dt
    x32 = x.cpu().numpy()
    mesh.close()
    disp = np.max(np.linalg.norm(x64 - scene.x0, axis=1))
    assert np.max(np.linalg.norm(x32 - x64, axis=1)) <= 1e-3 * disp
    assert abs(rep.energy - E64[-1]) <= 1e-6 * abs(E64[-1])
