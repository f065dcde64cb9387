"""Parity at the full 64^3-cube size (1,572,864 tets) and on the quadratic
and cubic benchmark boxes (about 137K DoF), in the launch configurations
that bench.py times.

The oracle cannot assemble the whole Hessian at this size in a test, so it
checks sampled block rows: for each sampled node, the oracle's element
derivatives of the node's incident elements are summed in element order into
the node's gradient row and Hessian block row, with inertia and Dirichlet, and
compared with the device's row.  The Newton step is checked through properties
that hold at any size, with the oracle's full float64 gradient and energy.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements, rest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL = 1e-4


@pytest.fixture(scope="module")
def symx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02156_amd import symx as s
    s.load()
    return s


@pytest.fixture(scope="module")
def c2():
    return sg.config_c2()


def _sample_nodes(scene, n, seed):
    """Interior, surface and fixed nodes, seeded."""
    rng = np.random.default_rng(seed)
    fixed = np.nonzero(scene.fixed)[0]
    free = np.nonzero(scene.fixed == 0)[0]
    return np.unique(np.concatenate([rng.choice(free, n - 16, replace=False),
                                     rng.choice(fixed, 16, replace=False),
                                     [0, scene.n_nodes - 1]]))


def _oracle_rows(scene, x, xt, dt, nodes, project=False):
    """Gradient rows and Hessian block rows {(i, j): 3x3} of the sampled nodes,
    from the oracle's element functions on the incident elements of every
    energy set, summed in (set, element) order (element Hessians projected to
    PSD, or SNH density Hessians filtered, as the assembly does with
    project=True / "filter")."""
    import dataclasses
    mass = rest.lumped_mass(scene)
    w = mass / dt ** 2
    fixed = scene.fixed.astype(bool)
    g = {int(i): np.zeros(3) for i in nodes}
    blocks = {int(i): {} for i in nodes}
    for es in scene.energies:
        conn = es.conn
        sel = np.nonzero(np.isin(conn, nodes).any(axis=1))[0]    # ascending element ids
        if sel.size == 0:
            continue
        sub = dataclasses.replace(es, conn=conn[sel], young_per_elem=None if es.young_per_elem
                                  is None else es.young_per_elem[sel])
        _, ge, He = elements.element_eval(sub, x, scene.X)
        k = conn.shape[1]
        if project == "filter" and es.kind == sg.SNH_TET4:
            mu, lam = rest.lame(rest.young_array(sub), sub.poisson)
            _, _, He = elements.snh_tet4_filtered(x[sub.conn], scene.X[sub.conn], mu, lam)
        elif project:
            He = assembly.project_psd(He.reshape(-1, 3 * k, 3 * k))
        ge = ge.reshape(-1, k, 3)
        He = He.reshape(-1, k, 3, k, 3)
        csel = conn[sel]
        for i in nodes:
            bi = blocks[int(i)]
            for e, a in np.argwhere(csel == i):                    # ascending element id
                g[int(i)] += ge[e, a]
                for b in range(k):
                    j = int(csel[e, b])
                    bi[j] = bi.get(j, np.zeros((3, 3))) + He[e, a, :, b, :]
    rows = {}
    for i in nodes:
        i = int(i)
        gi, bi = g[i], blocks[i]
        gi += w[i] * (x[i] - xt[i])
        bi[i] = bi.get(i, np.zeros((3, 3))) + w[i] * np.eye(3)
        if fixed[i]:
            gi[:] = 0.0
        for j in bi:
            if fixed[i] or fixed[j]:
                bi[j] = np.eye(3) if j == i else np.zeros((3, 3))
        rows[i] = (gi, bi)
    return rows


def _strained(scene, amp, seed):
    """x(t) plus U(-amp, amp)^3 on the free nodes (seeded): a strained state at
    which the elastic gradient is far from zero and element Hessians are
    indefinite, so projection and filtering change them."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amp, amp, size=scene.x0.shape)
    return scene.x0 + np.where(scene.fixed[:, None] == 1, 0.0, d)


def _check_sampled_rows(symx, scene, precision, n_nodes, seed, project=False, x=None):
    """Sampled gradient and Hessian block rows at x (default x(t)) against the
    oracle.  With projection, also checks that the oracle's projected rows
    differ from its raw rows (the projection acts at x)."""
    x = scene.x0 if x is None else x
    mesh = symx.Mesh(scene)
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    if project:
        flags |= symx.SYMX_PROJECT_FILTER if project == "filter" else symx.SYMX_PROJECT_PSD
    E, g, vals = mesh.assemble(x, xt, dt, flags, p)
    rp, ci, _ = mesh.pattern()
    V = vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3)
    gd = g.cpu().numpy()
    nodes = _sample_nodes(scene, n_nodes, seed=seed)
    ref = _oracle_rows(scene, x, xt, dt, nodes, project)
    if project:
        raw = _oracle_rows(scene, x, xt, dt, nodes, False)
        diff = max(np.abs(ref[i][1][j] - raw[i][1][j]).max() for i in ref for j in ref[i][1])
        scale = max(np.abs(raw[i][1][j]).max() for i in raw for j in raw[i][1])
        assert diff > 1e-3 * scale, (diff, scale)
    gerr = gmax = herr = hmax = 0.0
    for i, (go, blocks) in ref.items():
        cols = ci[rp[i]:rp[i + 1]]
        assert sorted(blocks) == list(cols)                        # row pattern
        gerr = max(gerr, np.abs(gd[i] - go).max())
        gmax = max(gmax, np.abs(go).max())
        for s_, j in enumerate(cols):
            herr = max(herr, np.abs(V[rp[i] + s_] - blocks[int(j)]).max())
            hmax = max(hmax, np.abs(blocks[int(j)]).max())
    assert herr <= tol * hmax
    assert gerr <= tol * max(gmax, 1e-300)
    E_ref = assembly.energy(scene, x, xt, dt)
    assert abs(E - E_ref) <= tol * abs(E_ref)
    mesh.close()


@pytest.fixture(scope="module")
def c2_strained(c2):
    """C2 positions plus U(+-20% of the cube edge) on the free nodes."""
    return _strained(c2, 0.2 * 0.01, 51)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c2_sampled_rows_match_oracle(symx, c2, c2_strained, precision):
    _check_sampled_rows(symx, c2, precision, 200, 41, x=c2_strained)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c2_rest_sampled_rows_match_oracle(symx, c2, precision):
    """At x(t) = X: zero elastic gradient, the rest stiffness."""
    _check_sampled_rows(symx, c2, precision, 60, 42)


@pytest.mark.parametrize("project", [True, "filter"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c2_projected_sampled_rows_match_oracle(symx, c2, c2_strained, precision, project):
    """Per-element PSD projection and the filtered SNH Hessian at full size, at
    a strained state where both change the element Hessians."""
    _check_sampled_rows(symx, c2, precision, 120, 45, project, x=c2_strained)


# The quadratic and cubic stretched boxes of the benchmark (about 137K DoF).
HIGH_ORDER_BOXES = {"quadratic": (sg.SNH_TET10, (17, 17, 18)),
                    "cubic": (sg.SNH_TET20, (11, 11, 13))}


@pytest.mark.parametrize("order", ["quadratic", "cubic"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_high_order_box_sampled_rows_match_oracle(symx, order, precision):
    kind, dims = HIGH_ORDER_BOXES[order]
    _check_sampled_rows(symx, sg.stretched_box_scene(kind, dims=dims), precision, 120, 43)


@pytest.mark.parametrize("order", ["quadratic", "cubic"])
def test_high_order_box_newton_step_f32_refined(symx, order):
    """One FP32-refined step on the benchmark box: the oracle's float64
    gradient at the result meets the Newton tolerance, the energy is the
    oracle's."""
    kind, dims = HIGH_ORDER_BOXES[order]
    scene = sg.stretched_box_scene(kind, dims=dims)
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=scene.dt,
                                                      precision=symx.SYMX_F32_REFINED))
    mesh.close()
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xh = x.cpu().numpy()
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, scene.dt, want_hess=False)["g"])
    assert rep.residual0 == pytest.approx(r0, rel=1e-10)
    r = np.linalg.norm(assembly.assemble(scene, xh, xt, scene.dt, want_hess=False)["g"])
    assert r <= 1.01e-6 * r0
    assert rep.energy == pytest.approx(assembly.energy(scene, xh, xt, scene.dt), rel=1e-10)


def test_c2_newton_step_f32_refined(symx, c2):
    """One FP32-refined step at full size: the oracle's float64 gradient at the
    result meets the Newton tolerance, and the reported energy is the oracle's."""
    scene = c2
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=scene.dt,
                                                      precision=symx.SYMX_F32_REFINED))
    mesh.close()
    assert st == 0, (symx.STATUS[st], rep.as_dict())
    xh = x.cpu().numpy()
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    r0 = np.linalg.norm(assembly.assemble(scene, scene.x0, xt, scene.dt, want_hess=False)["g"])
    assert rep.residual0 == pytest.approx(r0, rel=1e-10)
    r = np.linalg.norm(assembly.assemble(scene, xh, xt, scene.dt, want_hess=False)["g"])
    assert r <= 1.01e-6 * r0
    E_ref = assembly.energy(scene, xh, xt, scene.dt)
    assert rep.energy == pytest.approx(E_ref, rel=1e-10)
    assert np.allclose(v.cpu().numpy(), (xh - scene.x0) / scene.dt)


@pytest.mark.parametrize("kind", [sg.NH_TET4, sg.STVK_TET4, sg.FCR_TET4, sg.ARAP_TET4])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_material_box_sampled_rows_match_oracle(symx, kind, precision):
    """The other App. B materials on their benchmark box (40 x 40 x 60 cubes,
    576,000 tets; lagged rotations at the rest shape)."""
    _check_sampled_rows(symx, sg.stretched_box_scene(kind), precision, 80, 47)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_contact_scene_at_benchmark_size(symx, precision):
    """The contact benchmark (two stacked 32^3-cube blocks, 393,216 tets, 8,192
    candidates): energy and full gradient against the oracle, and every block
    of the contact matrix against the oracle's active contact blocks."""
    from oracle import contact
    scene = sg.contact_stack_scene(32, neighbors=True)
    cl = scene.contacts
    mesh = symx.Mesh(scene)
    mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
    dt = scene.dt
    xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    tol = F64_TOL if precision == "f64" else F32_TOL
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    E, g, _ = mesh.assemble(scene.x0, xt, dt, flags, p)
    ref = assembly.assemble(scene, scene.x0, xt, dt, want_hess=False)
    assert abs(E - ref["E"]) <= tol * abs(ref["E"])
    gd = g.cpu().numpy()
    assert np.abs(gd - ref["g"]).max() <= tol * np.abs(ref["g"]).max()
    # contact blocks: candidate element Hessians of the active candidates,
    # summed per node pair, Dirichlet applied
    _, _, Hc, act = contact.point_plane_barrier(scene.x0[cl.tuples], cl.kc, cl.dhat)
    assert 0 < act.sum() < act.size
    fixed = scene.fixed.astype(bool)
    want = {}
    for t, He in zip(cl.tuples[act], Hc[act]):
        for a in range(4):
            for b in range(4):
                key = (int(t[a]), int(t[b]))
                blk = np.zeros((3, 3)) if fixed[t[a]] or fixed[t[b]] else He[a, :, b, :]
                want[key] = want.get(key, np.zeros((3, 3))) + blk
    rp, ci, vals = mesh.contact_bsr(p)
    scale = max(np.abs(b).max() for b in want.values())
    err, seen = 0.0, set()
    for i in range(len(rp) - 1):
        for q in range(rp[i], rp[i + 1]):
            key = (i, int(ci[q]))
            seen.add(key)
            err = max(err, np.abs(vals[q] - want.get(key, np.zeros((3, 3)))).max())
    assert set(want) <= seen
    assert err <= tol * scale
    mesh.close()


@pytest.fixture(scope="module")
def c3():
    return sg.config_c3()


@pytest.mark.parametrize("project", [False, True, "filter"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c3_sampled_rows_match_oracle(symx, c3, precision, project):
    """C3 (512^2 cloth with membranes and hinges, and a 32^3-cube tet block):
    rows of cloth and block nodes, several element kinds per row, at a strained
    state (U(+-20% of the cloth spacing) on the free nodes); plain, with
    per-element PSD projection, and with the filtered SNH Hessian (membranes
    and hinges projected)."""
    x = _strained(c3, 0.2 / 512, 53)
    _check_sampled_rows(symx, c3, precision, 120, 49, project, x=x)



def _lanczos_smallest(matvec, v0, iters):
    """Smallest Ritz value of a symmetric operator (Lanczos with full
    reorthogonalisation, on the device) and the residual norm of its Ritz
    vector: an eigenvalue lies within that distance of the Ritz value."""
    n = v0.numel()
    Q = torch.zeros((iters + 1, n), dtype=torch.float64, device="cuda")
    Q[0] = v0 / torch.linalg.norm(v0)
    alpha, beta = [], []
    for k in range(iters):
        w = matvec(Q[k])
        a = torch.dot(w, Q[k])
        for _ in range(2):
            w = w - Q[:k + 1].T @ (Q[:k + 1] @ w)
        b = torch.linalg.norm(w)
        alpha.append(float(a))
        beta.append(float(b))
        Q[k + 1] = w / b
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    ev, V = np.linalg.eigh(T)
    return float(ev[0]), abs(beta[-1] * V[-1, 0])


def test_c4_step_endpoints_are_distinct_stationary_minima(symx):
    """C4 at 64^3 cubes, step 1 (dt 0.005) from the float64 state after step 0:
    float64 Newton with the forcing term capped at 0.5 and at 0.1 lands on
    two endpoints a centimetre or more apart.  Both are stationary (the
    oracle's float64 gradient meets the Newton tolerance) and minima (the
    smallest eigenvalue of the float64 Hessian on the free DoFs is positive),
    and the oracle's energy halfway between them lies above both (they sit in
    different basins), so the incremental potential of this violently
    compressed, stiffness-contrasted block has several local minima and the
    linear solver's path picks one; FP32-refined with the same forcing lands
    on the float64 endpoint."""
    scene = sg.config_c4(64)
    mesh = symx.Mesh(scene)

    def step(xs, vs, dt, **kw):
        x = torch.tensor(xs, dtype=torch.float64, device="cuda")
        v = torch.tensor(vs, dtype=torch.float64, device="cuda")
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, max_pcg=500, **kw))
        assert st == 0, (symx.STATUS[st], rep.as_dict())
        return x.cpu().numpy(), v.cpu().numpy(), rep

    x0, v0, rep0 = step(scene.x0, scene.v0, 0.01, precision=symx.SYMX_F64)
    dt = 0.005
    xa, _, ra = step(x0, v0, dt, precision=symx.SYMX_F64, max_halvings=0)
    xf, _, rf = step(x0, v0, dt, precision=symx.SYMX_F64, max_halvings=0, forcing_max=0.1)
    xq, _, rq = step(x0, v0, dt, precision=symx.SYMX_F32_REFINED, max_halvings=0,
                     forcing_max=0.1)
    assert np.max(np.linalg.norm(xa - xf, axis=1)) > 1e-2
    assert np.max(np.linalg.norm(xq - xf, axis=1)) < 1e-6
    xt = elements.x_tilde(x0, v0, dt, scene.gravity)
    rp, ci = assembly.pattern_fast(scene)
    # an energy barrier between the endpoints: different basins
    E_end = [assembly.assemble(scene, x, xt, dt, want_hess=False, row_ptr=rp, col_idx=ci)["E"]
             for x in (xa, xf)]
    E_mid = assembly.assemble(scene, 0.5 * (xa + xf), xt, dt, want_hess=False, row_ptr=rp,
                              col_idx=ci)["E"]
    assert E_mid > max(E_end) + 1e-9 * abs(E_mid), (E_end, E_mid)
    r0 = np.linalg.norm(assembly.assemble(scene, x0, xt, dt, want_hess=False, row_ptr=rp,
                                          col_idx=ci)["g"])
    N = scene.n_nodes
    br = torch.tensor(np.repeat(np.arange(N), np.diff(rp)), dtype=torch.int64, device="cuda")
    cc = torch.tensor(ci, dtype=torch.int64, device="cuda")
    free = torch.tensor(np.repeat(scene.fixed == 0, 3), device="cuda")
    xtd = torch.tensor(xt, dtype=torch.float64, device="cuda")
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    for x in (xa, xf):
        g = assembly.assemble(scene, x, xt, dt, want_hess=False, row_ptr=rp, col_idx=ci)["g"]
        assert np.linalg.norm(g) <= 1.01e-6 * r0
        _, _, vals = mesh.assemble(x, xtd, dt, flags, symx.SYMX_F64)
        rows = torch.cat([3 * br + r for r in range(3) for c in range(3)])
        cols = torch.cat([3 * cc + c for r in range(3) for c in range(3)])
        H = torch.sparse_coo_tensor(torch.stack([rows, cols]), vals.reshape(-1),
                                    (3 * N, 3 * N)).coalesce().to_sparse_csr()
        # Lanczos on S H S with S = diag(H)^(-1/2): the same inertia as H
        # (Sylvester's law) and a far smaller condition number
        dmask = br == cc
        d = torch.ones(3 * N, dtype=torch.float64, device="cuda")
        for r in range(3):
            d[3 * br[dmask] + r] = vals[4 * r][dmask]
        assert bool(torch.all(d > 0))
        sc = 1.0 / torch.sqrt(d)
        gen = torch.Generator(device="cuda").manual_seed(7)
        v = torch.randn(3 * N, dtype=torch.float64, device="cuda", generator=gen) * free
        lam, res = _lanczos_smallest(lambda q: sc * (H @ (sc * q)), v, 1500)
        assert lam > 0.0 and res < 0.5 * lam, (lam, res)
        del H
    mesh.close()
