"""Serving loop: concurrent time-step requests of differently sized scenes.

Each result must be the same alone and in the mix.  Every request's kernels
use fixed reduction orders on its own buffers, so the check is bitwise.
Admission must keep the admitted footprint within the memory budget.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import assembly, elements

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def symx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_02156_amd import symx as s
    s.load()
    return s


def _requests():
    reqs = [dict(n=n, young=y, seed=s) for n, y, s in
            [(4, 2e4, 11), (7, 1e5, 12), (5, 5e5, 13), (9, 1e5, 14), (6, 3e4, 15), (3, 1e6, 16)]]
    return [(r, sg.c5_request_scene(r)) for r in reqs]


def _run(symx, scenes, slots, budget=1 << 36, precision=0):
    srv = symx.symx_server_create(budget, slots)
    keep, tickets = [], []
    prm = symx.step_params(dt=0.01, precision=precision)
    for _, sc in scenes:
        desc, k = symx.scene_desc(sc)
        keep.append(k)
        tickets.append(symx.symx_server_submit(srv, desc, np.ascontiguousarray(sc.x0),
                                               np.ascontiguousarray(sc.v0), prm))
    out = []
    for t, (_, sc) in zip(tickets, scenes):
        x = np.zeros_like(sc.x0)
        v = np.zeros_like(sc.v0)
        st, rep, times = symx.symx_server_poll(srv, t, 1, x, v)
        out.append((st, rep.as_dict(), x, v, times))
    stats = symx.symx_server_get_stats(srv)
    symx.symx_server_destroy(srv)
    return out, stats


@pytest.mark.parametrize("precision", [0, 2])
def test_alone_equals_in_the_mix(symx, precision):
    scenes = _requests()
    alone = []
    for item in scenes:                           # one request at a time
        res, _ = _run(symx, [item], 1, precision=precision)
        alone.append(res[0])
    mix, stats = _run(symx, scenes, 4, precision=precision)   # all at once, 4 slots
    assert stats.completed == len(scenes)
    assert stats.peak_active >= 2                  # requests really overlapped
    for (sa, ra, xa, va, _), (sm, rm, xm, vm, _) in zip(alone, mix):
        assert sa == 0 and sm == 0
        assert np.array_equal(xa, xm) and np.array_equal(va, vm)
        assert ra["newton_iters"] == rm["newton_iters"] and ra["pcg_iters"] == rm["pcg_iters"]


def test_served_step_equals_direct_step_and_converges(symx):
    (req, sc), = _requests()[1:2]
    res, _ = _run(symx, [(req, sc)], 2)
    st, rep, x, v, times = res[0]
    assert st == 0 and all(times[i] <= times[i + 1] for i in range(4))
    mesh = symx.Mesh(sc)
    xd = torch.tensor(sc.x0, dtype=torch.float64, device="cuda")
    vd = torch.tensor(sc.v0, dtype=torch.float64, device="cuda")
    st2, rep2 = mesh.newton_step(xd, vd, symx.step_params(dt=0.01))
    mesh.close()
    assert st2 == 0
    assert np.array_equal(xd.cpu().numpy(), x)
    xt = elements.x_tilde(sc.x0, sc.v0, 0.01, sc.gravity)
    g = assembly.assemble(sc, x, xt, 0.01, want_hess=False)["g"]
    assert np.linalg.norm(g) <= 1.01e-6 * rep["residual0"]


def test_admission_respects_budget(symx):
    scenes = _requests()
    big = max((sc for _, sc in scenes), key=lambda sc: sc.n_nodes)
    # a budget that admits the largest request with little to spare
    res, stats = _run(symx, scenes, 6, budget=int(1.2 * _estimate(symx, big)))
    assert all(r[0] == 0 for r in res)
    assert stats.peak_bytes <= stats.budget_bytes
    assert stats.peak_active < len(scenes)         # the budget really bound


def _estimate(symx, scene, precision=0):
    desc, keep = symx.scene_desc(scene)
    return symx.symx_server_estimate_bytes(desc, precision)


def test_request_over_budget_is_rejected(symx):
    (_, sc), = _requests()[3:4]
    srv = symx.symx_server_create(1 << 20, 2)
    desc, k = symx.scene_desc(sc)
    with pytest.raises(symx.SymxError, match="BUDGET"):
        symx.symx_server_submit(srv, desc, np.ascontiguousarray(sc.x0),
                                np.ascontiguousarray(sc.v0), symx.step_params(dt=0.01))
    symx.symx_server_destroy(srv)


def test_many_concurrent_requests_all_succeed(symx):
    """Regression: with many slots on non-blocking streams, every request of a
    stream of small scenes must start from zeroed device flags and succeed."""
    rng = np.random.default_rng(21)
    scenes = [sg.c5_request_scene(dict(n=int(n), young=1e5, seed=int(s)))
              for n, s in zip(rng.integers(3, 9, size=40), rng.integers(0, 1 << 30, size=40))]
    res, stats = _run(symx, [(None, sc) for sc in scenes], 8, precision=2)
    assert [r[0] for r in res] == [0] * len(scenes)
    assert stats.completed == len(scenes) and stats.peak_active >= 2
    # the PCG chunks of concurrently solving requests shared launches
    assert stats.pcg_batches > 0 and stats.pcg_chunks > stats.pcg_batches
    # and each result is the direct step's, bit for bit
    prm = symx.step_params(dt=0.01, precision=2)
    for (st, rep, x, v, _), sc in list(zip(res, scenes))[:6]:
        mesh = symx.Mesh(sc)
        xd = torch.tensor(sc.x0, dtype=torch.float64, device="cuda")
        vd = torch.tensor(sc.v0, dtype=torch.float64, device="cuda")
        st2, rep2 = mesh.newton_step(xd, vd, prm)
        mesh.close()
        assert st2 == 0 and np.array_equal(xd.cpu().numpy(), x) and np.array_equal(vd.cpu().numpy(), v)


def test_resident_patterns_are_reused_and_give_identical_results(symx):
    """Requests that repeat a connectivity (same n, other material and
    perturbation) reuse the device-resident pattern; each result must equal
    the one of a fresh, uncached mesh bit for bit."""
    rng = np.random.default_rng(22)
    reqs = [dict(n=int(n), young=float(y), seed=int(s)) for n, y, s in
            zip([5, 6, 5, 5, 6, 4, 5, 6], rng.uniform(2e4, 5e5, 8), rng.integers(0, 1 << 30, 8))]
    scenes = [(r, sg.c5_request_scene(r)) for r in reqs]
    res, stats = _run(symx, scenes, 3, precision=2)
    assert stats.pattern_misses >= 3 and stats.pattern_hits >= 1
    assert stats.pattern_hits + stats.pattern_misses == len(scenes)
    prm = symx.step_params(dt=0.01, precision=2)
    for (st, rep, x, v, _), (_, sc) in zip(res, scenes):
        mesh = symx.Mesh(sc)
        xd = torch.tensor(sc.x0, dtype=torch.float64, device="cuda")
        vd = torch.tensor(sc.v0, dtype=torch.float64, device="cuda")
        st2, rep2 = mesh.newton_step(xd, vd, prm)
        mesh.close()
        assert st == 0 and st2 == 0
        assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(vd.cpu().numpy(), v)


def test_idle_patterns_are_evicted_under_a_tight_budget(symx):
    """With a budget that fits one request, cached patterns of other sizes must
    make room: every request still runs and the charge stays in the budget."""
    reqs = [dict(n=n, young=1e5, seed=30 + i) for i, n in enumerate([6, 4, 6, 5, 4, 6])]
    scenes = [(r, sg.c5_request_scene(r)) for r in reqs]
    budget = int(1.05 * max(_estimate(symx, sc, 2) for _, sc in scenes))
    res, stats = _run(symx, scenes, 2, budget=budget, precision=2)
    assert [r[0] for r in res] == [0] * len(scenes)
    assert stats.peak_bytes <= stats.budget_bytes
    assert stats.pattern_cache_bytes <= stats.budget_bytes


def test_quadratic_and_cubic_requests_served_like_direct_steps(symx):
    """Quadratic and cubic tet scenes in a mix with a linear one: each served
    step equals the same step taken directly on a mesh, bit for bit."""
    scenes = [(None, sg.tet_cube_scene(2, kind=sg.SNH_TET10, seed=21, perturb=0.05, vel_std=0.05)),
              (None, sg.tet_cube_scene(2, kind=sg.SNH_TET20, seed=22, perturb=0.05, vel_std=0.05)),
              _requests()[0]]
    res, stats = _run(symx, scenes, 3)
    assert stats.completed == 3
    for (_, sc), (st, rep, x, v, _) in zip(scenes, res):
        assert st == 0, rep
        mesh = symx.Mesh(sc)
        xd = torch.tensor(sc.x0, dtype=torch.float64, device="cuda")
        vd = torch.tensor(sc.v0, dtype=torch.float64, device="cuda")
        st2, _ = mesh.newton_step(xd, vd, symx.step_params(dt=0.01))
        mesh.close()
        assert st2 == 0
        assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(vd.cpu().numpy(), v)


def _served_peak(symx, scene, precision, project):
    """Device bytes the pool of a fresh one-slot server handed out at most
    while it served one step of `scene`."""
    srv = symx.symx_server_create(1 << 36, 1)
    desc, keep = symx.scene_desc(scene)
    # memory is what is measured: a few Newton iterations at the given dt
    # (plain float32 may stop short of the tolerance: NOT_CONVERGED, or
    # LINE_SEARCH with no halving allowed)
    prm = symx.step_params(dt=0.01, precision=precision, project=project, max_newton=20,
                           max_halvings=0)
    t = symx.symx_server_submit(srv, desc, np.ascontiguousarray(scene.x0),
                                np.ascontiguousarray(scene.v0), prm)
    x = np.zeros_like(scene.x0)
    v = np.zeros_like(scene.v0)
    st, rep, times = symx.symx_server_poll(srv, t, 1, x, v)
    stats = symx.symx_server_get_stats(srv)
    symx.symx_server_destroy(srv)
    return st, stats.peak_device_bytes


@pytest.mark.parametrize("name", ["snh", "cloth", "fcr", "tet10", "tet20"])
def test_estimate_bounds_the_device_memory_used(symx, name):
    """The footprint admission charges is an upper bound of the device memory
    a request really takes (mesh, pattern, Newton workspace, projection
    records), in every precision and projection mode."""
    scenes = {
        "snh": lambda: sg.tet_cube_scene(6, seed=21, perturb=0.1),
        "cloth": lambda: sg.cloth_scene(10, perturb=0.1),
        "fcr": lambda: sg.stretched_box_scene(sg.FCR_TET4, dims=(4, 4, 6)),
        "tet10": lambda: sg.tet_cube_scene(3, kind=sg.SNH_TET10, seed=22, perturb=0.05),
        "tet20": lambda: sg.tet_cube_scene(2, kind=sg.SNH_TET20, seed=23, perturb=0.05),
    }
    scene = scenes[name]()
    modes = [0] if name.startswith("tet1") or name.startswith("tet2") else [0, 1]
    if name == "snh":
        modes.append(2)
    for precision in (symx.SYMX_F64, symx.SYMX_F32, symx.SYMX_F32_REFINED):
        bound = _estimate(symx, scene, precision)
        for project in modes:
            st, peak = _served_peak(symx, scene, precision, project)
            assert symx.STATUS[st] in ("OK", "NOT_CONVERGED", "LINE_SEARCH"), (
                name, precision, project, symx.STATUS[st])
            assert 0 < peak <= bound, (name, precision, project, peak, bound)
