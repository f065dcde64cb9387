#!/usr/bin/env python3
"""Benchmark of the element-derivative / BSR-assembly / Newton hot path on one GPU.

Workload (default): a 64^3 grid of cubes, 6 Stable Neo-Hookean tets each
(1,572,864 tets, 274,625 nodes, 4,018,753 3x3 blocks), E = 1e5 Pa, nu = 0.4,
rho = 1000, bottom face fixed, x(t) = rest, v(t) ~ N(0, 0.1^2) m/s per
component (seed 2), dt = 0.01 s, gravity -9.81 z; Newton to 1e-6 relative
residual, block-Jacobi PCG at most 500 iterations.  All inputs are synthetic
and resident on the GPU before timing starts.

One step = one implicit-Euler time step through the whole path (assembly of
energy, gradient and BSR Hessian; PCG; float64 refinement; line search;
update) in the FP32-with-refinement mode.  The JSON line reports
  value        element evaluation + assembly throughput (Melem/s, FP32, no
               projection): device time of one full E + gradient + BSR Hessian
               evaluation, median over repetitions
  ms_per_step  FP32-refined Newton time step (K timed steps)
and, beside them, FP64 figures, projection-on figures, the roofline of the
dominant kernel (live HIP-event timing inside the timed steps) and the FP64
CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
IDLE_MS = 0.004  # PCG launches shorter than this found the solve converged


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, N, nnzb, n_elem, t_bytes):
    """Bytes the method itself must move per launch of a kernel (no staging,
    no index metadata beyond the matrix structure, gathers counted once)."""
    if kernel == "pcg_spmv":
        # values + column index + row pointer; z read; p, q read and written
        return (9 * t_bytes + 4) * nnzb + 4 * (N + 1) + 5 * 3 * t_bytes * N
    if kernel == "pcg_update":
        # Dinv (9), x rw, r rw, z w, p r, q r (3 each)
        return (9 + 6 + 6 + 3 + 3 + 3) * t_bytes * N
    if kernel in ("row_assemble_gH", "row_assemble_H"):
        out = 9 * t_bytes * nnzb + (24 * N if kernel == "row_assemble_gH" else 0)
        # connectivity, positions and rest positions (float64), masses, x_tilde, flags
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N + N + out
    if kernel == "row_assemble_g":
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N + N + 24 * N
    if kernel == "energy":
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N
    return None


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_c2_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2303_02156_amd", "csrc", "symx_kernels.hip")).read()
    a = src.find(f"// [traffic-hash-begin {kernel}]")
    e = src.find(f"// [traffic-hash-end {kernel}]")
    if a < 0 or e < 0:
        return None
    if hashlib.sha256(src[a:e].encode()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


# Generated functions the Stable Neo-Hookean row assembly and energy kernels run.
ROW_GEN_FUNCS = ("snh_tet4_row0_gHoff", "snh_tet4_row0_g", "snh_tet4_s_E")


def row_kernel_hash():
    """Hash of the row-assembly kernel source (its inputs gather and kind
    dispatch, and the kernels) and of the generated element functions it runs;
    the committed VALU record is tied to it."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2303_02156_amd", "csrc")
    src = open(os.path.join(csrc, "symx_kernels.hip")).read()
    h = hashlib.sha256()
    for region in ("row_inputs", "row_assemble"):
        a = src.find(f"// [valu-hash-begin {region}]")
        e = src.find(f"// [valu-hash-end {region}]")
        if a < 0 or e < 0:
            return None
        h.update(src[a:e].encode())
    gen = open(os.path.join(csrc, "generated", "symx_generated.h")).read()
    for fn in ROW_GEN_FUNCS:
        a = gen.find(f"void {fn}(")
        e = gen.find("\n}\n", a)
        if a < 0 or e < 0:
            return None
        h.update(gen[a:e].encode())
    return h.hexdigest()


def measured_valu():
    """Wave-level VALU instructions per FP32 g+H row-assembly launch from the
    committed rocprofv3 counter run, or None when the source changed since."""
    path = os.path.join(ROOT, "profiles", "row_assemble_c2_valu.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != row_kernel_hash():
        return None
    return rec["sq_insts_valu_per_launch"]


def census_ops(name):
    """Operation count of a generated element function (the generator's census)."""
    path = os.path.join(ROOT, "paper_2303_02156_amd", "csrc", "generated", "symx_generated_meta.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if f and f[0] == name:
            return int(f[-1])
    return None


def serving_bench(symx, torch, n_requests=256, rate=200.0, slots=8):
    """C5: Poisson arrivals of time-step requests; p50/p99 latency, throughput."""
    import numpy as np

    import scenegen as sg
    reqs = sg.config_c5_requests(n_requests, rate)
    scenes = [sg.c5_request_scene(r) for r in reqs]
    descs = [symx.scene_desc(sc) for sc in scenes]
    prm = symx.step_params(dt=0.01, precision=symx.SYMX_F32_REFINED)
    est = [symx.symx_server_estimate_bytes(d, symx.SYMX_F32_REFINED) for d, _ in descs]
    n_tets = sum(sc.n_elements() for sc in scenes)
    free, _ = torch.cuda.mem_get_info()

    def run(budget, n_slots, paced):
        srv = symx.symx_server_create(budget, n_slots)
        t0 = time.perf_counter()
        tickets = []
        for r, (desc, _), sc in zip(reqs, descs, scenes):
            if paced:
                delay = t0 + r["t"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.append(symx.symx_server_submit(srv, desc, np.ascontiguousarray(sc.x0),
                                                   np.ascontiguousarray(sc.v0), prm))
        lat, ends, ok, statuses, failed, phases = [], [], 0, {}, [], []
        for i, tk in enumerate(tickets):
            st, rep, times = symx.symx_server_poll(srv, tk, 1)
            ok += int(st == 0)
            name = symx.STATUS.get(st, str(st))
            statuses[name] = statuses.get(name, 0) + 1
            if st != 0:
                failed.append({"request": i, "n": reqs[i]["n"], "status": name,
                               "error": symx.load().symx_last_error().decode(),
                               "report": {k: rep.as_dict()[k] for k in
                                          ("newton_iters", "pcg_iters", "dt_halvings")}})
            lat.append(times[4] - times[0])
            ends.append(times[4])
            phases.append(np.diff(times))
        stats = symx.symx_server_get_stats(srv)
        symx.symx_server_destroy(srv)
        span_s = max(ends) / 1e3  # server creation to last completion
        return {"budget_gb": round(budget / 1e9, 3), "slots": n_slots,
                "arrivals": "poisson 200/s" if paced else "all at t=0",
                "completed_ok": ok, "statuses": statuses, "failed": failed[:8],
                "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "requests_per_s": round(float(len(reqs) / span_s), 2),
                "melem_steps_per_s": round(float(n_tets / span_s / 1e6), 3),
                "peak_active": stats.peak_active, "peak_gb": round(stats.peak_bytes / 1e9, 3),
                "pattern_cache": {"hits": stats.pattern_hits, "misses": stats.pattern_misses},
                "mean_phase_ms": dict(zip(("queued", "setup", "step", "teardown"),
                                          [round(float(v), 2) for v in np.mean(phases, axis=0)]))}

    out = {"requests": n_requests, "tets_total": n_tets,
           "n_range": [min(r["n"] for r in reqs), max(r["n"] for r in reqs)]}
    out["full_budget"] = run(int(0.8 * free), slots, True)
    log(f"serving full budget: {out['full_budget']}")
    binding = sum(sorted(est)[-3:])
    out["binding_budget"] = run(binding, slots, True)
    log(f"serving binding budget: {out['binding_budget']}")
    out["sequential"] = run(int(0.8 * free), 1, False)
    log(f"serving sequential: {out['sequential']}")
    return out


def trajectory(symx, torch, scene, precision, steps, dt):
    """Run `steps` implicit-Euler steps; returns (x, v, reports, ms per step)."""
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    prm = symx.step_params(dt=dt, precision=precision, max_pcg=500)
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        st, rep = mesh.newton_step(x, v, prm)
        reps.append(rep.as_dict())
        log(f"  {scene.name} {symx.STATUS[st]} step {k}: newton {rep.newton_iters} pcg "
            f"{rep.pcg_iters} halvings {rep.dt_halvings} {rep.ms_total:.1f} ms")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = (x.cpu().numpy(), v.cpu().numpy(), reps, ms)
    mesh.close()
    return out


def precision_c4(symx, torch, n=64, steps=10):
    """C4: stiff heterogeneous compressed grid, FP32-refined against all-FP64.

    The FP64 run chooses the time steps (with dt halving); the FP32-refined
    runs reuse that exact dt sequence with halving off, so both reach the same
    simulated times:
      per step   from each FP64 state, one FP32-refined step, compared with the
                 next FP64 state (relative to that step's displacement)
      trajectory FP32-refined from the start along the same dt sequence,
                 compared after all steps (relative to the total displacement)
    """
    import numpy as np

    import scenegen as sg
    scene = sg.config_c4(n)
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    states, dts, E64, ms64 = [(scene.x0.copy(), scene.v0.copy())], [], [], []
    p64 = symx.step_params(dt=scene.dt, precision=symx.SYMX_F64, max_pcg=500)
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = mesh.newton_step(x, v, p64)
        torch.cuda.synchronize()
        ms64.append((time.perf_counter() - t0) * 1e3)
        if st != 0:
            mesh.close()
            return {"error": f"FP64 step {k} failed: {symx.STATUS[st]}"}
        dts.append(rep.dt_used)
        E64.append(rep.energy)
        states.append((x.cpu().numpy(), v.cpu().numpy()))
        log(f"  C4 f64 step {k}: dt {rep.dt_used:.3g} newton {rep.newton_iters} "
            f"pcg {rep.pcg_iters} halvings {rep.dt_halvings}")

    def step32(xs, vs, dt):
        xd = torch.tensor(xs, dtype=torch.float64, device="cuda")
        vd = torch.tensor(vs, dtype=torch.float64, device="cuda")
        prm = symx.step_params(dt=dt, precision=symx.SYMX_F32_REFINED, max_pcg=500,
                               max_halvings=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = mesh.newton_step(xd, vd, prm)
        torch.cuda.synchronize()
        return st, rep, xd.cpu().numpy(), vd.cpu().numpy(), (time.perf_counter() - t0) * 1e3

    local_pos, local_E, ms32 = [], [], []
    for k in range(steps):
        st, rep, x32, _, ms = step32(states[k][0], states[k][1], dts[k])
        ms32.append(ms)
        if st != 0:
            local_pos.append(float("inf"))
            continue
        local_pos.append(float(np.max(np.linalg.norm(x32 - states[k + 1][0], axis=1))))
        local_E.append((rep.energy - E64[k]) / abs(E64[k]))
    xs, vs = states[0]
    traj_ok, fail_at = True, None
    for k in range(steps):
        st, rep, xs, vs, _ = step32(xs, vs, dts[k])
        if st != 0:
            traj_ok, fail_at = False, k
            break
    out = {"workload": f"C4: {n}^3 cubes x 6 SNH tets, E ~ logU(1e4, 1e7) seed 4, 30% "
                       "compression, top and bottom fixed, dt 0.01 with halving",
           "steps": steps, "dt_sequence": dts,
           "ms_per_step": {"f32_refined_same_dt": round(float(np.mean(ms32)), 3),
                           "f64": round(float(np.mean(ms64)), 3)},
           "per_step_max_abs_position_error_m": max(local_pos),
           "per_step_max_rel_position_error": max(local_pos) / float(
               max(np.max(np.linalg.norm(s[0] - scene.x0, axis=1)) for s in states[1:])),
           "per_step_max_rel_energy_error": max(abs(e) for e in local_E) if local_E else None,
           "per_step_abs_position_error_m": [float("%.3g" % e) for e in local_pos],
           "per_step_signed_rel_energy_diff_f32r_minus_f64": [float("%.3g" % e) for e in local_E],
           "per_step_note": "steps whose energies differ reached different local minima of the "
                            "non-convex incremental potential (both meet the 1e-6 residual test)",
           "trajectory_converged": traj_ok, "trajectory_failed_at_step": fail_at}
    if traj_ok:
        xT = states[-1][0]
        disp = np.max(np.linalg.norm(xT - scene.x0, axis=1))
        out["trajectory_max_rel_position_error"] = float(
            np.max(np.linalg.norm(xs - xT, axis=1)) / disp)
        out["trajectory_max_abs_position_error_m"] = float(np.max(np.linalg.norm(xs - xT, axis=1)))
        out["trajectory_rel_energy_error"] = float(abs(rep.energy - E64[-1]) / abs(E64[-1]))
    mesh.close()
    return out


def mixed_c3(symx, torch, steps=20):
    """C3: 512^2 cloth (membrane + hinges) beside a 32^3 tet block, FP32-refined."""
    import scenegen as sg
    scene = sg.config_c3()
    mesh = symx.Mesh(scene)
    info = mesh.info
    dt = scene.dt
    import numpy as np
    xt = torch.tensor(scene.x0 + dt * scene.v0 + dt * dt * np.asarray(scene.gravity)[None, :],
                      dtype=torch.float64, device="cuda")
    x0 = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x0)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    ms = []
    for r in range(13):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        symx.symx_assemble_bsr(mesh.handle, x0.data_ptr(), xt.data_ptr(), dt, flags,
                               symx.SYMX_F32, g.data_ptr())
        b.record()
        b.synchronize()
        if r >= 3:
            ms.append(a.elapsed_time(b))
    asm_ms = statistics.median(ms)
    mesh.close()
    n_elem = scene.n_elements()
    _, _, reps, ms_step = trajectory(symx, torch, scene, symx.SYMX_F32_REFINED, steps, dt)
    return {"workload": "C3: 512^2 cloth (524,288 StVK triangles, 785,408 hinges, pinned edge) "
                        "+ 32^3-cube SNH block (196,608 tets), dt 1/60",
            "elements": n_elem, "nnzb": int(info.nnzb),
            "assembly_ms_f32": round(asm_ms, 4),
            "melem_per_s_f32": round(n_elem / (asm_ms * 1e-3) / 1e6, 2),
            "steps": steps, "ms_per_step_f32_refined": round(ms_step, 3),
            "newton_iters": sum(r["newton_iters"] for r in reps),
            "pcg_iters": sum(r["pcg_iters"] for r in reps),
            "all_converged": all(r["status"] == 0 for r in reps),
            "dt_halvings": sum(r["dt_halvings"] for r in reps)}


# Evaluation + assembly per Newton iteration on the material-comparison box
# (Sec. 6.1: 307,623 DoF), in ms on the reference CPU (application timings
# table); context only, another machine.
PAPER_MATERIAL_MS = {"arap": 38.79, "fcr": 35.40, "stvk": 37.85, "nh": 35.83, "snh": 35.10}


def materials_bench(symx, torch, reps=10):
    """The five tet materials on the stretched box (40 x 40 x 60 cubes, 576,000
    tets, 102,541 nodes): one E+g+H assembly in FP32 and FP64 (device events,
    median of reps), and one FP32-refined Newton step from the stretched state
    with lagged rotations taken at x(t)."""
    import numpy as np
    import scenegen as sg
    kinds = {"snh": sg.SNH_TET4, "nh": sg.NH_TET4, "stvk": sg.STVK_TET4, "fcr": sg.FCR_TET4,
             "arap": sg.ARAP_TET4}
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    out = {}
    for name, kind in kinds.items():
        scene = sg.stretched_box_scene(kind)
        mesh = symx.Mesh(scene)
        n_elem = scene.n_elements()
        dt = scene.dt
        x0 = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
        v0 = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
        xt = torch.tensor(scene.x0 + dt * scene.v0 + dt * dt * np.asarray(scene.gravity)[None, :],
                          dtype=torch.float64, device="cuda")
        g = torch.empty_like(x0)
        mesh.update_rotations(x0)
        row = {"elements": n_elem, "dof": 3 * scene.n_nodes}
        for pname, prec in (("f32", symx.SYMX_F32), ("f64", symx.SYMX_F64)):
            ms = []
            for r in range(reps + 3):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                symx.symx_assemble_bsr(mesh.handle, x0.data_ptr(), xt.data_ptr(), dt, flags, prec,
                                       g.data_ptr())
                b.record()
                b.synchronize()
                if r >= 3:
                    ms.append(a.elapsed_time(b))
            m = statistics.median(ms)
            row[f"assembly_ms_{pname}"] = round(m, 4)
            row[f"melem_per_s_{pname}"] = round(n_elem / (m * 1e-3) / 1e6, 2)
        x = x0.clone()
        v = v0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, precision=symx.SYMX_F32_REFINED,
                                                          max_pcg=500))
        torch.cuda.synchronize()
        row.update({"newton_ms_f32_refined": round((time.perf_counter() - t0) * 1e3, 2),
                    "status": symx.STATUS[st], "newton_iters": rep.newton_iters,
                    "pcg_iters": rep.pcg_iters,
                    "rel_residual": rep.residual / max(rep.residual0, 1e-300),
                    "paper_cpu_ms_per_newton_iter": PAPER_MATERIAL_MS[name]})
        mesh.close()
        log(f"material {name}: {row}")
        out[name] = row
    return {"workload": "stretched box: 40x40x60 cubes x 6 tets (576,000 tets, 307,623 DoF), "
                        "E=1e4 nu=0.3, top face held at 1.2x height, +-1% noise (seed 6), "
                        "dt=0.01",
            "materials": out}


# Higher-order tets on the stretched box: the paper's per-Newton-iteration
# evaluation + assembly time of its 137K-DoF stretched cube with quadratic and
# cubic elements (simulation benchmark table, SymX column) and its
# single-element E+g+H time of such a tet (single element benchmark table),
# CPU, ms and us; context only, another machine.
PAPER_TET10_MS_PER_ITER = 24.3
PAPER_TET10_US_PER_ELEM = 5.91
PAPER_TET20_MS_PER_ITER = 52.9
PAPER_TET20_US_PER_ELEM = 64.13

# order -> (kind, box dims in cubes, points of the rule, row functions with
# the number of local nodes that use each, paper numbers)
HIGH_ORDER = {
    "quadratic": dict(kind=7, k=10, dims=(17, 17, 18), pts=4, rule="4-point rule",
                      rows=(("snh_tet10_row0_gHoff", 4), ("snh_tet10_row4_gHoff", 6)),
                      paper=(PAPER_TET10_MS_PER_ITER, PAPER_TET10_US_PER_ELEM)),
    "cubic": dict(kind=8, k=20, dims=(11, 11, 13), pts=11, rule="Keast 11-point rule",
                  rows=(("snh_tet20_row0_gHoff", 4), ("snh_tet20_row4_gHoff", 12),
                        ("snh_tet20_row19_gHoff", 4)),
                  paper=(PAPER_TET20_MS_PER_ITER, PAPER_TET20_US_PER_ELEM)),
}


def high_order_bench(symx, torch, order, reps=10):
    """Quadratic or cubic SNH tets (Eq. 12) on a stretched box of about 137K
    DoF (quadratic: 17 x 17 x 18 cubes, 31,212 tets, 135,975 DoF; cubic:
    11 x 11 x 13 cubes, 9,438 tets, 138,720 DoF): one E+g+H assembly in FP32
    and FP64 (device events, median of reps) and one FP32-refined Newton step.
    row_ops_per_elem counts the generated operations of the row functions the
    assembly evaluates (every node of every element at every point)."""
    import numpy as np
    import scenegen as sg
    cfg = HIGH_ORDER[order]
    scene = sg.stretched_box_scene(cfg["kind"], dims=cfg["dims"])
    mesh = symx.Mesh(scene)
    n_elem = scene.n_elements()
    dt = scene.dt
    x0 = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v0 = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    xt = torch.tensor(scene.x0 + dt * scene.v0 + dt * dt * np.asarray(scene.gravity)[None, :],
                      dtype=torch.float64, device="cuda")
    g = torch.empty_like(x0)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    nx, ny, nz = cfg["dims"]
    out = {"workload": f"stretched box of {order} SNH tets: {nx}x{ny}x{nz} cubes x 6 "
                       f"tet{cfg['k']} ({n_elem} elements, {3 * scene.n_nodes} DoF), E=1e4 "
                       "nu=0.3, top face held at 1.2x height, +-1% noise (seed 6), dt=0.01, "
                       + cfg["rule"],
           "elements": n_elem, "dof": 3 * scene.n_nodes, "nnzb": int(mesh.info.nnzb)}
    for pname, prec in (("f32", symx.SYMX_F32), ("f64", symx.SYMX_F64)):
        ms = []
        for r in range(reps + 3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            symx.symx_assemble_bsr(mesh.handle, x0.data_ptr(), xt.data_ptr(), dt, flags, prec,
                                   g.data_ptr())
            b.record()
            b.synchronize()
            if r >= 3:
                ms.append(a.elapsed_time(b))
        m = statistics.median(ms)
        out[f"assembly_ms_{pname}"] = round(m, 4)
        out[f"ns_per_elem_{pname}"] = round(m * 1e6 / n_elem, 2)
    row_ops = [census_ops(name) for name, _ in cfg["rows"]]
    if all(row_ops):
        ops = cfg["pts"] * sum(o * n for o, (_, n) in zip(row_ops, cfg["rows"]))
        out["row_ops_per_elem"] = ops
        for pname in ("f32", "f64"):
            out[f"achieved_tflops_{pname}"] = round(
                ops * n_elem / (out[f"assembly_ms_{pname}"] * 1e-3) / 1e12, 2)
    x = x0.clone()
    v = v0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, precision=symx.SYMX_F32_REFINED,
                                                      max_pcg=500))
    torch.cuda.synchronize()
    out.update({"newton_ms_f32_refined": round((time.perf_counter() - t0) * 1e3, 2),
                "status": symx.STATUS[st], "newton_iters": rep.newton_iters,
                "pcg_iters": rep.pcg_iters,
                "rel_residual": rep.residual / max(rep.residual0, 1e-300),
                "paper_cpu_ms_per_newton_iter": cfg["paper"][0],
                "paper_cpu_us_per_elem": cfg["paper"][1]})
    mesh.close()
    log(f"{order} tets: {out}")
    return out


def contact_bench(symx, torch, n=32, reps=10):
    """Conditional point-plane barrier on two stacked SNH cubes of n^3 6-tet
    cubes: every node of the upper bottom face against both triangles of the
    lower top-face cells around it (about 8 candidates per node, half of them
    within d_hat).  E+g+H assembly with and without contacts (FP32, device
    events, median of reps), the contact kernels' device times, and one
    FP32-refined Newton step."""
    import numpy as np
    import scenegen as sg
    scene = sg.contact_stack_scene(n, neighbors=True)
    cl = scene.contacts
    mesh = symx.Mesh(scene)
    dt = scene.dt
    x0 = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v0 = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    xt = torch.tensor(scene.x0 + dt * scene.v0 + dt * dt * np.asarray(scene.gravity)[None, :],
                      dtype=torch.float64, device="cuda")
    g = torch.empty_like(x0)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET

    def timed():
        ms = []
        for r in range(reps + 3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            symx.symx_assemble_bsr(mesh.handle, x0.data_ptr(), xt.data_ptr(), dt, flags,
                                   symx.SYMX_F32, g.data_ptr())
            b.record()
            b.synchronize()
            if r >= 3:
                ms.append(a.elapsed_time(b))
        return statistics.median(ms)
    t_plain = timed()
    # the candidate list is handed over again at every time step (dynamic
    # topology): time repeated calls after two warm-up calls
    set_ms_all = []
    for r in range(7):
        t0 = time.perf_counter()
        mesh.set_contacts(cl.tuples, cl.kc, cl.dhat)
        set_ms_all.append((time.perf_counter() - t0) * 1e3)
    set_ms = statistics.median(set_ms_all[2:])
    t_contact = timed()
    mesh.profile(True)
    for _ in range(3):
        mesh.assemble(x0, xt, dt, flags, symx.SYMX_F32, grad_out=g)
    kt = {k: round(v[1] / max(v[0], 1), 5) for k, v in mesh.kernel_times().items()
          if k.startswith("contact")}
    mesh.profile(False)
    cview = symx.symx_mesh_get_contact_bsr(mesh.handle, symx.SYMX_F32)
    x = x0.clone()
    v = v0.clone()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, rep = mesh.newton_step(x, v, symx.step_params(dt=dt, precision=symx.SYMX_F32_REFINED,
                                                      max_pcg=500))
    torch.cuda.synchronize()
    out = {"workload": f"two stacked {n}^3-cube SNH blocks ({scene.n_elements()} tets), "
                       f"{cl.tuples.shape[0]} point-plane candidates (k_c {cl.kc}, d_hat "
                       f"{cl.dhat}), upper block moving down at 0.05 m/s, dt 0.01",
           "candidates": int(cl.tuples.shape[0]), "contact_blocks": int(cview.nnzb),
           "set_contacts_ms": round(set_ms, 3),
           "set_contacts_first_call_ms": round(set_ms_all[0], 2),
           "assembly_ms_f32_without_contacts": round(t_plain, 4),
           "assembly_ms_f32_with_contacts": round(t_contact, 4),
           "contact_kernel_avg_ms": kt,
           "newton_ms_f32_refined": round((time.perf_counter() - t1) * 1e3, 2),
           "status": symx.STATUS[st], "newton_iters": rep.newton_iters, "pcg_iters": rep.pcg_iters}
    mesh.close()
    log(f"contacts: {out}")
    return out


def cpu_baseline(seconds_target=10.0):
    """FP64 numpy oracle: eval + assembly (E, g, BSR) of a 24^3 cube of the same
    workload recipe, repeated until ~seconds_target of CPU work."""
    import numpy as np

    import scenegen as sg
    from oracle import assembly, elements
    n = 24
    s = sg.tet_cube_scene(n, h=0.01, seed=2, perturb=0.0, vel_std=0.1)
    rp, ci = assembly.pattern_fast(s)
    xt = elements.x_tilde(s.x0, s.v0, 0.01, s.gravity)
    ne = s.energies[0].conn.shape[0]
    times = []
    cpu0 = time.process_time()
    w0 = time.perf_counter()
    while sum(times) < seconds_target and len(times) < 8:
        t = time.perf_counter()
        assembly.assemble(s, xt, xt, 0.01, row_ptr=rp, col_idx=ci)
        times.append(time.perf_counter() - t)
    wall = time.perf_counter() - w0
    cores = max(1, round((time.process_time() - cpu0) / wall))
    med = statistics.median(times)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(ne / med / 1e6, 5), "unit": "Melem/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"FP64 numpy oracle, E+g+BSR assembly of a 24^3-cube grid ({ne} tets, "
                      f"same material/state recipe), median of {len(times)} passes "
                      f"({sum(times):.1f} s); host {model or platform.processor()}, "
                      f"{os.cpu_count()} logical CPUs visible"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=64, help="cubes per side")
    ap.add_argument("--asm-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64-newton", action="store_true")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving workload")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-materials", action="store_true")
    ap.add_argument("--no-quadratic", action="store_true")
    ap.add_argument("--no-cubic", action="store_true")
    ap.add_argument("--no-contacts", action="store_true")
    ap.add_argument("--only", choices=["c3", "c4", "materials", "quadratic", "cubic", "contacts"],
                    help="run only this extra workload")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run plain 512 MiB device copies first (byte-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} / WORLD_SIZE {world} "
              "is not supported (the multi-GPU sharding is a design note, not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen as sg
    from paper_2303_02156_amd import symx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    symx.load()
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(symx, torch)}), flush=True)
        return
    if args.only == "c3":
        print(json.dumps({"c3": mixed_c3(symx, torch)}), flush=True)
        return
    if args.only == "c4":
        print(json.dumps({"c4": precision_c4(symx, torch)}), flush=True)
        return
    if args.only == "materials":
        print(json.dumps({"materials": materials_bench(symx, torch)}), flush=True)
        return
    if args.only in HIGH_ORDER:
        print(json.dumps({args.only: high_order_bench(symx, torch, args.only)}), flush=True)
        return
    if args.only == "contacts":
        print(json.dumps({"contacts": contact_bench(symx, torch)}), flush=True)
        return
    if args.calib_copy:
        # a plain copy kernel of known size: 512 MiB read + 512 MiB written per launch
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copies done (4 x 512 MiB)")
    scene = sg.config_c2(args.n)
    n_elem = scene.n_elements()
    log(f"scene {scene.name}: {scene.n_nodes} nodes, {n_elem} tets")
    t = time.perf_counter()
    mesh = symx.Mesh(scene)
    setup_s = time.perf_counter() - t
    N, nnzb = mesh.info.n_nodes, mesh.info.nnzb
    log(f"mesh setup {setup_s:.2f} s, nnzb {nnzb}, batches {mesh.info.n_batches}")
    dt = scene.dt
    xt_np = scene.x0 + dt * scene.v0 + dt * dt * np.asarray(scene.gravity)[None, :]
    x0 = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v0 = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    xt = torch.tensor(xt_np, dtype=torch.float64, device="cuda")
    g = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET

    # ---- element evaluation + assembly throughput --------------------------
    def time_assembly(precision, fl, reps):
        for _ in range(3):
            mesh.assemble(x0, xt, dt, fl, precision, grad_out=g)
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            symx.symx_assemble_bsr(mesh.handle, x0.data_ptr(), xt.data_ptr(), dt, fl, precision,
                                   g.data_ptr())
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return statistics.median(ms)

    melem = {}
    asm_ms = {}
    for name, prec in (("f32", symx.SYMX_F32), ("f64", symx.SYMX_F64)):
        m = time_assembly(prec, flags, args.asm_reps)
        asm_ms[name] = m
        melem[name] = n_elem / (m * 1e-3) / 1e6
        log(f"eval+assembly {name}: {m:.3f} ms -> {melem[name]:.1f} Melem/s")
    if not args.no_projection:
        for name, prec, fl in (("f32_project", symx.SYMX_F32, symx.SYMX_PROJECT_PSD),
                               ("f64_project", symx.SYMX_F64, symx.SYMX_PROJECT_PSD),
                               ("f32_filter", symx.SYMX_F32, symx.SYMX_PROJECT_FILTER),
                               ("f64_filter", symx.SYMX_F64, symx.SYMX_PROJECT_FILTER)):
            m = time_assembly(prec, flags | fl, 5)
            asm_ms[name] = m
            melem[name] = n_elem / (m * 1e-3) / 1e6
            log(f"eval+assembly {name}: {m:.3f} ms -> {melem[name]:.2f} Melem/s")
    # per-kernel split of FP32 assemblies (device time per launch)
    mesh.profile(True)
    n_prof = 5
    for _ in range(n_prof):
        mesh.assemble(x0, xt, dt, flags, symx.SYMX_F32, grad_out=g)
    asm_kernels = mesh.kernel_times()
    mesh.profile(False)
    roofline_asm = None
    kt_gh = asm_kernels.get("row_assemble_gH")
    kt_e = asm_kernels.get("energy")
    ops_elem = census_ops("snh_tet4_EgH")
    if kt_gh and kt_gh[0] and kt_e and ops_elem:
        t_gh = kt_gh[1] / kt_gh[0]
        t_e = kt_e[1] / n_prof
        achieved = ops_elem * n_elem / ((t_gh + t_e) * 1e-3) / 1e12
        peak = 78.6
        valu = measured_valu()
        executed = [census_ops("snh_tet4_row0_gHoff"), census_ops("snh_tet4_s_E")]
        roofline_asm = {
            "kernel": "row_assemble_gH + energy (FP32 E, g, H)", "bound": "alu",
            "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "peak_note": "FP32 vector without packed math (packed FP32 is disabled): "
                         "256 CU x 64 lanes x 2.4 GHz x 2 (FMA)",
            "algorithmic_ops_per_elem": ops_elem,
            "executed_ops_per_elem": (4 * executed[0] + executed[1]) if all(executed) else None,
            "avg_ms": round(t_gh + t_e, 5),
            "valu_issue_frac": (round(valu / (t_gh * 1e-3 * 256 * 2.4e9), 3)
                                if valu else None),
        }
        log(f"assembly ALU roofline: {roofline_asm}")

    # ---- Newton time steps -----------------------------------------------------
    def run_steps(precision, K, W, profile):
        x = x0.clone()
        v = v0.clone()
        prm = symx.step_params(dt=dt, precision=precision, max_pcg=500)
        for k in range(W):
            st, rep = mesh.newton_step(x, v, prm)
            log(f"warmup step {k}: status {symx.STATUS[st]} newton {rep.newton_iters} "
                f"pcg {rep.pcg_iters} {rep.ms_total:.1f} ms")
        if profile:
            mesh.profile(True)
        reps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            st, rep = mesh.newton_step(x, v, prm)
            reps.append(rep.as_dict())
            log(f"step {k}: status {symx.STATUS[st]} newton {rep.newton_iters} pcg "
                f"{rep.pcg_iters} refine {rep.refinements} halvings {rep.dt_halvings} "
                f"res {rep.residual:.3e}/{rep.residual0:.3e} {rep.ms_total:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = None
        if profile:
            # launches enqueued past PCG convergence only test a flag (< 4 us)
            kt = {"busy": mesh.kernel_times(min_ms=IDLE_MS), "all": mesh.kernel_times()}
            mesh.profile(False)
        return wall * 1e3 / K, reps, kt

    # timed run without per-kernel events (they add host work to every launch)
    ms_f32r, reps_f32r, _ = run_steps(symx.SYMX_F32_REFINED, args.steps, args.warmup, False)
    log(f"newton f32_refined: {ms_f32r:.2f} ms/step")
    # replay of the identical (deterministic) step sequence with per-kernel
    # start/stop events; kernel device times feed the roofline
    ms_prof, reps_prof, ktimes = run_steps(symx.SYMX_F32_REFINED, args.steps, args.warmup, True)
    log(f"newton f32_refined with kernel events: {ms_prof:.2f} ms/step")
    same = [(a["newton_iters"], a["pcg_iters"]) for a in reps_f32r] == \
        [(a["newton_iters"], a["pcg_iters"]) for a in reps_prof]
    ms_f64, reps_f64 = None, None
    if not args.no_f64_newton:
        ms_f64, reps_f64, _ = run_steps(symx.SYMX_F64, args.steps, args.warmup, False)
        log(f"newton f64: {ms_f64:.2f} ms/step")

    # ---- roofline of the dominant kernel (live HIP-event timing) --------------
    busy, allk = ktimes["busy"], ktimes["all"]
    kname, (launches, total_ms) = max(busy.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / max(launches, 1)
    t_bytes = 4
    nbytes = algorithmic_bytes(kname, N, nnzb, n_elem, t_bytes)
    roofline = {"kernel": kname, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": None, "launches": launches,
                "avg_ms": round(avg_ms, 5), "algorithmic_bytes": nbytes,
                "idle_launches": allk[kname][0] - launches,
                "idle_ms": round(allk[kname][1] - total_ms, 3),
                "share_of_step_time": round(allk[kname][1] / (ms_f32r * args.steps), 4),
                "timing": "hipExtLaunchKernelGGL start/stop events in a replay of the timed "
                          "steps (identical iteration counts: %s)" % same}
    if nbytes:
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        roofline["achieved"] = round(ach, 1)
        roofline["frac"] = round(ach / HBM_PEAK_GBS, 4)
    if args.n == 64:
        roofline["traffic"] = measured_traffic(kname)
    kernels = {}
    for k, (n, ms) in sorted(allk.items(), key=lambda kv: -kv[1][1]):
        nb_, msb = busy.get(k, (0, 0.0))
        d = {"launches": n, "total_ms": round(ms, 3), "busy_launches": nb_,
             "busy_avg_ms": round(msb / max(nb_, 1), 5)}
        b_ = algorithmic_bytes(k, N, nnzb, n_elem, t_bytes)
        if b_ and nb_:
            d["busy_gbs"] = round(b_ / (msb / nb_ * 1e-3) / 1e9, 1)
        kernels[k] = d

    c4 = None if args.no_c4 else precision_c4(symx, torch)
    if c4:
        log(f"c4: {c4}")
    c3 = None if args.no_c3 else mixed_c3(symx, torch)
    if c3:
        log(f"c3: {c3}")
    materials = None if args.no_materials else materials_bench(symx, torch)
    quadratic = None if args.no_quadratic else high_order_bench(symx, torch, "quadratic")
    cubic = None if args.no_cubic else high_order_bench(symx, torch, "cubic")
    contacts = None if args.no_contacts else contact_bench(symx, torch)

    serving = None
    if not args.no_serving:
        log("serving (256 requests, Poisson 200/s)...")
        serving = serving_bench(symx, torch)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)...")
        cpu = cpu_baseline()
        log(f"cpu baseline {cpu['value']} Melem/s")

    def summary(reps):
        if not reps:
            return None
        return {"newton_iters": sum(r["newton_iters"] for r in reps),
                "pcg_iters": sum(r["pcg_iters"] for r in reps),
                "refinements": sum(r["refinements"] for r in reps),
                "dt_halvings": sum(r["dt_halvings"] for r in reps),
                "all_converged": all(r["status"] == 0 for r in reps),
                "max_rel_residual": max(r["residual"] / max(r["residual0"], 1e-300) for r in reps)}

    out = {
        "metric": "elem eval+assembly Melem/s, Newton step ms FP32-refined vs FP64; p99 latency",
        "value": round(melem["f32"], 2),
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_f32r, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C2: {args.n}^3-cube grid x 6 Stable Neo-Hookean tets "
                               f"({n_elem} tets, {N} nodes, {nnzb} 3x3 blocks), E=1e5 nu=0.4, "
                               "v~N(0,0.1) seed 2, dt=0.01, Newton rtol 1e-6, PCG<=500",
                   "precision": "FP32 element kernels/SpMV/PCG, FP64 energies, gradient, "
                                "residual and refinement"},
        "melem_per_s": {k: round(v, 3) for k, v in melem.items()},
        "assembly_ms": {k: round(v, 4) for k, v in asm_ms.items()},
        "assembly_kernels_f32": {k: {"launches": n, "ms": round(ms, 4)}
                                 for k, (n, ms) in asm_kernels.items()},
        "newton_step_ms_with_kernel_events": round(ms_prof, 3),
        "newton_step_ms": {"f32_refined": round(ms_f32r, 3),
                           "f64": None if ms_f64 is None else round(ms_f64, 3)},
        "newton_f32_refined": summary(reps_f32r),
        "newton_f64": summary(reps_f64),
        "p99_latency_ms": None if serving is None else serving["full_budget"]["p99_ms"],
        "serving": serving,
        "c4_precision": c4,
        "c3_mixed": c3,
        "materials": materials,
        "quadratic_tets": quadratic,
        "cubic_tets": cubic,
        "contacts": contacts,
        "mesh_setup_s": round(setup_s, 3),
        "kernels_f32_refined_steps": kernels,
        "roofline": roofline,
        "roofline_assembly": roofline_asm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
