"""The allocation-free assembly entry point (symx_assemble_bsr_noalloc) against
symx_assemble_bsr, through the C-ABI: energy, gradient and BSR values are the
same bit for bit (the same kernels, the same summation order), on two calls in
a row, the second on a smaller mesh, so that the shared scratch array is
reused with a smaller input."""
import numpy as np
import pytest

import scenegen as sg
from oracle import elements

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def symx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02156_amd import symx as s
    s.load()
    return s


def _flags(symx):
    return symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET


def _reference(symx, mesh, x, xt, dt, flags, precision):
    """symx_assemble_bsr, the existing entry point."""
    E, g, vals = mesh.assemble(x, xt, dt, flags, precision)
    return E, g.cpu().numpy(), None if vals is None else vals.cpu().numpy()


def _noalloc(symx, mesh, x, xt, dt, flags, precision):
    dtype = torch.float64 if precision == symx.SYMX_F64 else torch.float32
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    xtd = None if xt is None else torch.tensor(xt, dtype=torch.float64, device="cuda")
    g = torch.full((mesh.N, 3), np.nan, dtype=torch.float64, device="cuda")
    vals = torch.full((9, mesh.info.nnzb), np.nan, dtype=dtype, device="cuda")
    st, E = symx.symx_assemble_bsr_noalloc(mesh.handle, xd.data_ptr(),
                                           None if xtd is None else xtd.data_ptr(), dt, flags,
                                           precision, g.data_ptr(), vals.data_ptr())
    torch.cuda.synchronize()
    return st, E, g.cpu().numpy(), vals.cpu().numpy()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_matches_assemble_bsr_twice(symx, precision):
    p = symx.SYMX_F64 if precision == "f64" else symx.SYMX_F32
    flags = _flags(symx)
    # first call: C1 (6,000 tets); second: a 4^3-cube box (384 tets)
    for scene in (sg.config_c1(), sg.tet_cube_scene(4, seed=3, perturb=0.05)):
        mesh = symx.Mesh(scene)
        dt = scene.dt
        xt = elements.x_tilde(scene.x0, scene.v0, dt, scene.gravity)
        E0, g0, v0 = _reference(symx, mesh, scene.x0, xt, dt, flags, p)
        st, E1, g1, v1 = _noalloc(symx, mesh, scene.x0, xt, dt, flags, p)
        assert symx.STATUS[st] == "OK"
        assert E1 == E0
        assert np.array_equal(g1, g0)
        assert np.array_equal(v1, v0)
        mesh.close()


def test_noalloc_other_flags_and_kinds(symx):
    """Gradient only, energy only, no inertia, the filtered SNH Hessian, and a
    mesh of tets, membranes and hinges."""
    scene = sg.tet_cube_scene(3, seed=7, perturb=0.2)
    mesh = symx.Mesh(scene)
    xt = elements.x_tilde(scene.x0, scene.v0, scene.dt, scene.gravity)
    E_, G_, H_ = symx.SYMX_EVAL_E, symx.SYMX_EVAL_GRAD, symx.SYMX_EVAL_HESS
    for flags, with_xt in ((E_ | G_, True), (E_, False), (E_ | G_ | H_, False),
                           (E_ | G_ | H_ | symx.SYMX_PROJECT_FILTER | symx.SYMX_DIRICHLET, True)):
        x_t = xt if with_xt else None
        E0, g0, v0 = _reference(symx, mesh, scene.x0, x_t, scene.dt, flags, symx.SYMX_F64)
        st, E1, g1, v1 = _noalloc(symx, mesh, scene.x0, x_t, scene.dt, flags, symx.SYMX_F64)
        assert symx.STATUS[st] == "OK", flags
        assert E1 == E0
        if flags & G_:
            assert np.array_equal(g1, g0)
        if flags & H_:
            assert np.array_equal(v1, v0)
    mesh.close()
    c = sg.cloth_scene(6, perturb=0.2)
    s = sg.tet_cube_scene(2, seed=5, perturb=0.1)
    N = s.n_nodes
    es = [s.energies[0]] + [sg.EnergySet(e.kind, e.conn + N, young=e.young, poisson=e.poisson,
                                         thickness=e.thickness, bend_kb=e.bend_kb,
                                         density=e.density) for e in c.energies]
    mixed = sg.Scene("mixed", np.concatenate([s.X, c.X]), es,
                     np.concatenate([s.fixed, c.fixed]), np.concatenate([s.x0, c.x0]),
                     np.zeros((N + c.n_nodes, 3)))
    mesh = symx.Mesh(mixed)
    xt = elements.x_tilde(mixed.x0, mixed.v0, 0.01, mixed.gravity)
    for p in (symx.SYMX_F64, symx.SYMX_F32):
        E0, g0, v0 = _reference(symx, mesh, mixed.x0, xt, 0.01, _flags(symx), p)
        st, E1, g1, v1 = _noalloc(symx, mesh, mixed.x0, xt, 0.01, _flags(symx), p)
        assert symx.STATUS[st] == "OK"
        assert E1 == E0 and np.array_equal(g1, g0) and np.array_equal(v1, v0)
    mesh.close()


def test_noalloc_rejections_and_nonfinite(symx):
    scene = sg.tet_cube_scene(2, seed=1)
    mesh = symx.Mesh(scene)
    flags = _flags(symx)
    xd = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    g = torch.empty((mesh.N, 3), dtype=torch.float64, device="cuda")
    vals = torch.empty((9, mesh.info.nnzb), dtype=torch.float64, device="cuda")
    h = mesh.handle
    # Hessian without a values array; per-element PSD projection (records)
    st, _ = symx.symx_assemble_bsr_noalloc(h, xd.data_ptr(), None, 0.0, flags, symx.SYMX_F64,
                                           g.data_ptr(), None)
    assert symx.STATUS[st] == "INVALID_ARG"
    st, _ = symx.symx_assemble_bsr_noalloc(h, xd.data_ptr(), None, 0.0,
                                           flags | symx.SYMX_PROJECT_PSD, symx.SYMX_F64,
                                           g.data_ptr(), vals.data_ptr())
    assert symx.STATUS[st] == "INVALID_ARG"
    # a non-finite position is reported, and the next call starts from a
    # cleared flag
    xbad = xd.clone()
    xbad[5, 1] = float("nan")
    st, _ = symx.symx_assemble_bsr_noalloc(h, xbad.data_ptr(), None, 0.0, flags, symx.SYMX_F64,
                                           g.data_ptr(), vals.data_ptr())
    assert symx.STATUS[st] == "NONFINITE"
    st, E = symx.symx_assemble_bsr_noalloc(h, xd.data_ptr(), None, 0.0, flags, symx.SYMX_F64,
                                           g.data_ptr(), vals.data_ptr())
    assert symx.STATUS[st] == "OK" and np.isfinite(E)
    mesh.close()
    # meshes with contacts
    cs = sg.contact_stack_scene(2)
    mesh = symx.Mesh(cs)
    mesh.set_contacts(cs.contacts.tuples, cs.contacts.kc, cs.contacts.dhat)
    xd = torch.tensor(cs.x0, dtype=torch.float64, device="cuda")
    g = torch.empty((mesh.N, 3), dtype=torch.float64, device="cuda")
    vals = torch.empty((9, mesh.info.nnzb), dtype=torch.float64, device="cuda")
    st, _ = symx.symx_assemble_bsr_noalloc(mesh.handle, xd.data_ptr(), None, 0.0, flags,
                                           symx.SYMX_F64, g.data_ptr(), vals.data_ptr())
    assert symx.STATUS[st] == "INVALID_ARG"
    mesh.close()
