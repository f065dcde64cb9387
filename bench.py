#!/usr/bin/env python3
"""Benchmark of the element-derivative / BSR-assembly / Newton hot path on one GPU.

Workload (default): a 64^3 grid of cubes, 6 Stable Neo-Hookean tets each
(1,572,864 tets, 274,625 nodes, 4,018,753 3x3 blocks), E = 1e5 Pa, nu = 0.4,
rho = 1000, bottom face fixed, x(t) = rest, v(t) ~ N(0, 0.1^2) m/s per
component (seed 2), dt = 0.01 s, gravity -9.81 z; Newton to 1e-6 relative
residual, block-Jacobi PCG at most 500 iterations.  All inputs are synthetic
and resident on the GPU before timing starts.

One step = one implicit-Euler time step through the whole path (assembly of
energy, gradient and BSR Hessian; PCG; line search; update) in float64, the
paper's precision.  The JSON line reports
  value        element evaluation + assembly throughput (Melem/s, FP64, no
               projection): device time of one full E + gradient + BSR Hessian
               evaluation, median over repetitions
  ms_per_step  FP64 Newton time step (K timed steps)
  roofline     the FP64 PCG SpMV, the dominant kernel of the step (live
               HIP-event timing in a replay of the timed steps)
and, beside them, FP32 and FP32-with-refinement figures, projection-on
figures, the FP32 SpMV (Infinity-Cache resident, labelled "mall"), the
assembly's ALU roofline, and the FP64 CPU oracle timed on all host cores of
the GPU's CPU share and on one core.  The other workloads (C3, C4, beam,
materials, higher-order tets, contacts, serving) are logged to stderr and,
with --details, written to a JSON file.
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
        # the symmetric matrix's half (blocks (i, j), j <= i: values and
        # column index) + row pointer; z read; p, q read and written
        nnzl = (nnzb + N) // 2
        return (9 * t_bytes + 4) * nnzl + 4 * (N + 1) + 5 * 3 * t_bytes * N
    if kernel == "pcg_update":
        # Dinv (6: the upper triangle of each symmetric block inverse),
        # x rw, r rw, z w, p r, q r (3 each)
        return (6 + 6 + 6 + 3 + 3 + 3) * t_bytes * N
    if kernel in ("row_assemble_gH", "row_assemble_H"):
        out = 9 * t_bytes * nnzb + (24 * N if kernel == "row_assemble_gH" else 0)
        # connectivity, positions and rest positions (float64), masses, x_tilde, flags
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N + N + out
    if kernel == "row_assemble_g":
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N + N + 24 * N
    if kernel == "energy":
        return 16 * n_elem + 24 * N + 24 * N + 8 * N + 24 * N
    return None


def measured_traffic(kernel, label):
    """HBM bytes per launch of kernel<label> (label "float" or "double") from
    the committed rocprofv3 counter runs, or None when the kernel source
    changed since the counters were taken."""
    import hashlib
    tag = {"float": "f32", "double": "f64"}[label]
    path = os.path.join(ROOT, "profiles", f"{kernel}_{tag}_c2_traffic.json")
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
                "pcg_batches": stats.pcg_batches, "pcg_chunks": stats.pcg_chunks,
                "chunks_per_batch": round(stats.pcg_chunks / max(stats.pcg_batches, 1), 2),
                "mean_phase_ms": dict(zip(("queued", "setup", "step", "teardown"),
                                          [round(float(v), 2) for v in np.mean(phases, axis=0)]))}

    out = {"requests": n_requests, "tets_total": n_tets,
           "n_range": [min(r["n"] for r in reqs), max(r["n"] for r in reqs)]}
    out["full_budget"] = run(int(0.8 * free), slots, True)
    log(f"serving full budget: {out['full_budget']}")
    binding = sum(sorted(est)[-3:])
    out["binding_budget"] = run(binding, slots, True)
    log(f"serving binding budget: {out['binding_budget']}")
    # saturated: every request queued at t = 0, so the slots stay full and
    # the run measures the capacity of the batched server
    out["saturated"] = run(int(0.8 * free), slots, False)
    log(f"serving saturated: {out['saturated']}")
    out["sequential"] = run(int(0.8 * free), 1, False)
    log(f"serving sequential: {out['sequential']}")
    return out


def trajectory(symx, torch, scene, precision, steps, dt, profile_steps=0, max_pcg=500):
    """Run `steps` implicit-Euler steps; returns (x, v, reports, ms per step),
    and with profile_steps > 0 also {kernel: (launches, device ms)} of that
    many more steps run with per-launch events (after the timed ones)."""
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
    prm = symx.step_params(dt=dt, precision=precision, max_pcg=max_pcg)
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
    if profile_steps:
        mesh.profile(True)
        preps = []
        for k in range(profile_steps):
            st, rep = mesh.newton_step(x.clone(), v.clone(), prm)
            preps.append(rep.as_dict())
        kt = mesh.kernel_times()
        mesh.profile(False)
        out = out + ((kt, preps),)
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
    # steps where the two runs landed apart: the incremental potential has
    # several local minima there and the Newton path picks one (the forcing
    # term decides it in float64 alone); with the forcing term capped at 0.1
    # both precisions take the same path, which gives the error on one branch
    same_branch = []
    for k, dpos in enumerate(local_pos):
        if not (dpos > 1e-4):
            continue
        pair = []
        for prec in (symx.SYMX_F64, symx.SYMX_F32_REFINED):
            xd = torch.tensor(states[k][0], dtype=torch.float64, device="cuda")
            vd = torch.tensor(states[k][1], dtype=torch.float64, device="cuda")
            st, rep = mesh.newton_step(xd, vd, symx.step_params(dt=dts[k], precision=prec,
                                                                max_pcg=500, max_halvings=0,
                                                                forcing_max=0.1))
            pair.append((st, rep.energy, xd.cpu().numpy()))
        same_branch.append({
            "step": k, "default_forcing_abs_position_diff_m": float("%.4g" % dpos),
            "default_forcing_energies_f64_f32r": [E64[k], E64[k] + local_E[k] * abs(E64[k])]
            if k < len(local_E) else None,
            "forcing_0.1_status": [symx.STATUS[pair[0][0]], symx.STATUS[pair[1][0]]],
            "forcing_0.1_energies_f64_f32r": [pair[0][1], pair[1][1]],
            "forcing_0.1_abs_position_diff_m": float(
                "%.4g" % np.max(np.linalg.norm(pair[0][2] - pair[1][2], axis=1)))})
    # trajectories on one branch: both precisions with the forcing term
    # capped at 0.1 (the FP64 run chooses the time steps, FP32-refined replays
    # them)
    def traj(prec, dts_in):
        xd = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
        vd = torch.tensor(scene.v0, dtype=torch.float64, device="cuda")
        used, E = [], None
        for k in range(steps):
            kw = dict(max_halvings=8) if dts_in is None else dict(max_halvings=0)
            st, rep = mesh.newton_step(xd, vd, symx.step_params(
                dt=scene.dt if dts_in is None else dts_in[k], precision=prec, max_pcg=500,
                forcing_max=0.1, **kw))
            if st != 0:
                return None, used, None
            used.append(rep.dt_used)
            E = rep.energy
        return xd.cpu().numpy(), used, E
    x64b, dts_b, E64b = traj(symx.SYMX_F64, None)
    x32b, _, E32b = traj(symx.SYMX_F32_REFINED, dts_b) if x64b is not None else (None, None, None)
    traj_b = None
    if x64b is not None and x32b is not None:
        disp_b = np.max(np.linalg.norm(x64b - scene.x0, axis=1))
        traj_b = {"dt_sequence": dts_b,
                  "max_rel_position_error": float(np.max(np.linalg.norm(x32b - x64b, axis=1)) / disp_b),
                  "max_abs_position_error_m": float(np.max(np.linalg.norm(x32b - x64b, axis=1))),
                  "rel_energy_error": float(abs(E32b - E64b) / abs(E64b))}
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
           "same_branch": same_branch,
           "trajectory_forcing_0.1": traj_b,
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
    _, _, reps, ms_step, (kt, preps) = trajectory(symx, torch, scene, symx.SYMX_F32_REFINED,
                                                  steps, dt, profile_steps=2)
    # where a step's device time goes (2 more steps with per-launch events):
    # the solve (SpMV, update, refinement residual) against the assembly,
    # energies and the rest
    solve = ("pcg_spmv", "pcg_update", "pcg_init", "residual64", "accumulate")
    assembly_k = ("row_assemble_gH", "row_assemble_H", "row_assemble_g", "round_values")
    tot = sum(t for _, t in kt.values())
    t_solve = sum(kt[k][1] for k in solve if k in kt)
    t_asm = sum(kt[k][1] for k in assembly_k if k in kt)
    newton = sum(r["newton_iters"] for r in reps)
    pcg = sum(r["pcg_iters"] for r in reps)
    # the same steps with the PCG cap at 2000: the capped solves (cap 500)
    # return inexact directions, and Newton then needs many more iterations
    _, _, reps2k, ms_step2k = trajectory(symx, torch, scene, symx.SYMX_F32_REFINED, steps, dt,
                                         max_pcg=2000)
    newton2k = sum(r["newton_iters"] for r in reps2k)
    pcg2k = sum(r["pcg_iters"] for r in reps2k)
    return {"workload": "C3: 512^2 cloth (524,288 StVK triangles, 785,408 hinges, pinned edge) "
                        "+ 32^3-cube SNH block (196,608 tets), dt 1/60",
            "elements": n_elem, "nnzb": int(info.nnzb),
            "assembly_ms_f32": round(asm_ms, 4),
            "melem_per_s_f32": round(n_elem / (asm_ms * 1e-3) / 1e6, 2),
            "steps": steps, "ms_per_step_f32_refined": round(ms_step, 3),
            "newton_iters": newton, "pcg_iters": pcg,
            "pcg_iters_per_solve": round(pcg / max(newton, 1), 1),
            "pcg_cap": 500,
            "all_converged": all(r["status"] == 0 for r in reps),
            "dt_halvings": sum(r["dt_halvings"] for r in reps),
            "device_ms_split_2_steps": {
                "solve": round(t_solve, 2), "assembly": round(t_asm, 2),
                "other": round(tot - t_solve - t_asm, 2),
                "newton_iters": sum(r["newton_iters"] for r in preps),
                "pcg_iters": sum(r["pcg_iters"] for r in preps)},
            "pcg_cap_2000": {"ms_per_step_f32_refined": round(ms_step2k, 3),
                             "newton_iters": newton2k, "pcg_iters": pcg2k,
                             "pcg_iters_per_solve": round(pcg2k / max(newton2k, 1), 1),
                             "all_converged": all(r["status"] == 0 for r in reps2k),
                             "dt_halvings": sum(r["dt_halvings"] for r in reps2k)}}


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


_CPU = {}


def _cpu_init(n):
    """Worker set-up of the all-core oracle baseline: the scene, its pattern and
    the prediction x_tilde (setup, not timed)."""
    import scenegen as sg
    from oracle import assembly, elements
    s = sg.tet_cube_scene(n, h=0.01, seed=2, perturb=0.0, vel_std=0.1)
    rp, ci = assembly.pattern_fast(s)
    _CPU.update(scene=s, rp=rp, ci=ci, xt=elements.x_tilde(s.x0, s.v0, 0.01, s.gravity))


def _cpu_chunk(rng):
    """One worker's share: the oracle's assembly of elements [lo, hi) (no inertia,
    no Dirichlet) at the predicted positions; returns the touched slice of the
    gradient rows and of the block values."""
    import copy

    import numpy as np

    from oracle import assembly
    lo, hi = rng
    s, rp, ci, xt = _CPU["scene"], _CPU["rp"], _CPU["ci"], _CPU["xt"]
    sub = copy.copy(s)
    es = copy.copy(s.energies[0])
    es.conn = es.conn[lo:hi]
    sub.energies = [es]
    a = assembly.assemble(sub, xt, None, None, dirichlet=False, row_ptr=rp, col_idx=ci)
    n0, n1 = int(es.conn.min()), int(es.conn.max()) + 1
    b0, b1 = int(rp[n0]), int(rp[n1])
    return a["E"], n0, a["g"][n0:n1], b0, a["vals"][b0:b1]


def cpu_baseline(seconds_target=10.0):
    """The FP64 numpy oracle timed on the host, before the GPU is touched:
    - one core: the oracle's E + g + BSR assembly of a 24^3-cube grid (82,944
      tets) of the workload recipe, repeated for about seconds_target;
    - all cores: a 32^3-cube grid (196,608 tets) split into one contiguous
      element range per worker process (the CPU share of one GPU, at most 16
      workers); each runs the same oracle assembly on its range and the parent
      adds the touched row and block slices, then the inertia term and the
      Dirichlet rows (the rest of the oracle's assembly).  Wall time per pass,
      median of several passes after one warm-up."""
    import multiprocessing as mp

    import numpy as np

    import scenegen as sg
    from oracle import assembly, elements
    from oracle.rest import lumped_mass

    def host_model():
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
        except OSError:
            pass
        return platform.processor()

    # one core
    n1 = 24
    s = sg.tet_cube_scene(n1, h=0.01, seed=2, perturb=0.0, vel_std=0.1)
    rp, ci = assembly.pattern_fast(s)
    xt = elements.x_tilde(s.x0, s.v0, 0.01, s.gravity)
    ne1 = s.energies[0].conn.shape[0]
    times = []
    while sum(times) < seconds_target and len(times) < 8:
        t = time.perf_counter()
        assembly.assemble(s, xt, xt, 0.01, row_ptr=rp, col_idx=ci)
        times.append(time.perf_counter() - t)
    one = ne1 / statistics.median(times) / 1e6

    # all cores of the GPU's CPU share
    n_all = 32
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(16, avail))
    sa = sg.tet_cube_scene(n_all, h=0.01, seed=2, perturb=0.0, vel_std=0.1)
    rpa, cia = assembly.pattern_fast(sa)
    xta = elements.x_tilde(sa.x0, sa.v0, 0.01, sa.gravity)
    nea = sa.energies[0].conn.shape[0]
    m = lumped_mass(sa)
    fixed = sa.fixed.astype(bool)
    rows = np.repeat(np.arange(sa.n_nodes), np.diff(rpa))
    kill = fixed[rows] | fixed[cia]
    diag = np.nonzero(rows == cia)[0]
    cuts = np.linspace(0, nea, workers + 1).astype(int)
    ranges = [(int(cuts[i]), int(cuts[i + 1])) for i in range(workers)]
    ctx = mp.get_context("fork")
    times_all = []
    with ctx.Pool(workers, initializer=_cpu_init, initargs=(n_all,)) as pool:
        pool.map(_cpu_chunk, ranges)  # warm-up
        while sum(times_all) < seconds_target / 2 and len(times_all) < 8:
            t = time.perf_counter()
            parts = pool.map(_cpu_chunk, ranges)
            g = np.zeros((sa.n_nodes, 3))
            vals = np.zeros((cia.size, 3, 3))
            E = 0.0
            for Ep, n0, gp, b0, vp in parts:
                E += Ep
                g[n0:n0 + gp.shape[0]] += gp
                vals[b0:b0 + vp.shape[0]] += vp
            Ei, gi, w = elements.inertia(xta, xta, m, 0.01)
            E += float(np.sum(Ei))
            g += gi
            vals[diag] += w[:, None, None] * np.eye(3)[None]
            g[fixed] = 0.0
            vals[kill] = 0.0
            vals[diag[fixed]] = np.eye(3)
            times_all.append(time.perf_counter() - t)
    allc = nea / statistics.median(times_all) / 1e6
    return {"value": round(allc, 4), "unit": "Melem/s", "cores": workers, "kind": "oracle",
            "value_1core": round(one, 5),
            "sample": f"FP64 numpy oracle, E+g+BSR assembly (eval+assembly, as the GPU value): "
                      f"{workers} worker processes on a {n_all}^3-cube grid ({nea} tets), "
                      f"median of {len(times_all)} passes; one core on a {n1}^3-cube grid "
                      f"({ne1} tets), median of {len(times)} passes; host {host_model()}, "
                      f"{avail} CPUs available"}


def c1_oracle_newton():
    """The oracle's Newton step on C1 (block-Jacobi PCG, the device's control
    logic), wall time on one core; run before the GPU is touched."""
    import scenegen as sg
    from oracle import newton
    s = sg.config_c1()
    t = time.perf_counter()
    ok, x, rep = newton.newton_solve(s, s.x0, s.v0, s.dt, newton.StepParams(dt=s.dt))
    return {"ms": round((time.perf_counter() - t) * 1e3, 1), "ok": ok,
            "newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"], "x": x}


def c1_newton_vs_oracle(symx, torch, oracle_c1):
    """One C1 Newton step on the device (FP64 and FP32-refined, mean of 10 from
    x(t)) beside the oracle's (one core), with the largest position difference."""
    import numpy as np

    import scenegen as sg
    s = sg.config_c1()
    mesh = symx.Mesh(s)
    out = {"workload": "C1: 10^3 cubes x 6 SNH tets (6000 tets), one implicit-Euler step",
           "oracle_ms_1core": oracle_c1["ms"], "oracle_newton_iters": oracle_c1["newton_iters"],
           "oracle_pcg_iters": oracle_c1["pcg_iters"]}
    for name, prec in (("f64", symx.SYMX_F64), ("f32_refined", symx.SYMX_F32_REFINED)):
        ms = []
        for k in range(11):
            x = torch.tensor(s.x0, dtype=torch.float64, device="cuda")
            v = torch.tensor(s.v0, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, rep = mesh.newton_step(x, v, symx.step_params(dt=s.dt, precision=prec))
            torch.cuda.synchronize()
            if k:
                ms.append((time.perf_counter() - t) * 1e3)
        out[f"device_ms_{name}"] = round(float(np.mean(ms)), 3)
        out[f"device_newton_iters_{name}"] = rep.newton_iters
        out[f"max_abs_position_diff_to_oracle_m_{name}"] = float(
            "%.3g" % np.max(np.abs(x.cpu().numpy() - oracle_c1["x"])))
    mesh.close()
    return out


def beam_bench(symx, torch, reps=10):
    """The linear-tet beam of the simulation benchmark table: a k x k x 3k beam of
    6-tet cubes with k = 24 (25 * 25 * 73 nodes = 136,875 DoF, 248,832 tets),
    Stable Neo-Hookean E = 1e4 Pa, nu = 0.3, bottom fixed, top stretched 20%
    (the stretched-box recipe).  FP64 and FP32 eval+assembly (device events,
    median of reps) and one Newton step per precision, with the paper's CPU
    figures (another machine: context)."""
    import statistics as st_

    import scenegen as sg
    scene = sg.stretched_box_scene(sg.SNH_TET4, dims=(24, 24, 72), young=1e4, poisson=0.3)
    mesh = symx.Mesh(scene)
    x = torch.tensor(scene.x0, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x)
    flags = symx.SYMX_EVAL_E | symx.SYMX_EVAL_GRAD | symx.SYMX_EVAL_HESS | symx.SYMX_DIRICHLET
    out = {"workload": "24x24x72-cube SNH beam (136875 DoF, 248832 tets), E 1e4, nu 0.3, "
                       "stretched 20%, bottom and top fixed",
           "paper_cpu_ms": {"eval_assembly_per_newton_iter": 14.8, "pcg_per_newton_iter": 29.8,
                            "hardware": "Threadripper PRO 5975WX, 32 threads, FP64"}}
    for name, prec in (("f64", symx.SYMX_F64), ("f32", symx.SYMX_F32)):
        for _ in range(3):
            mesh.assemble(x, None, 0.0, flags, prec, grad_out=g)
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            symx.symx_assemble_bsr(mesh.handle, x.data_ptr(), None, 0.0, flags, prec, g.data_ptr())
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        out[f"assembly_ms_{name}"] = round(st_.median(ms), 4)
    for name, prec in (("f64", symx.SYMX_F64), ("f32_refined", symx.SYMX_F32_REFINED)):
        xs = x.clone()
        vs = torch.zeros_like(xs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, rep = mesh.newton_step(xs, vs, symx.step_params(dt=scene.dt, precision=prec))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        out[f"newton_{name}"] = {"status": symx.STATUS[st], "ms": round(ms, 2),
                                 "newton_iters": rep.newton_iters, "pcg_iters": rep.pcg_iters,
                                 "pcg_ms_per_newton_iter": round(rep.ms_pcg / max(rep.newton_iters, 1), 3)}
    mesh.close()
    log(f"beam: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=64, help="cubes per side")
    ap.add_argument("--asm-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32-newton", action="store_true")
    ap.add_argument("--no-beam", action="store_true")
    ap.add_argument("--details", default=None,
                    help="also write every section's figures to this JSON file")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving workload")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-materials", action="store_true")
    ap.add_argument("--no-quadratic", action="store_true")
    ap.add_argument("--no-cubic", action="store_true")
    ap.add_argument("--no-contacts", action="store_true")
    ap.add_argument("--only", choices=["c3", "c4", "materials", "quadratic", "cubic", "contacts",
                                       "beam"],
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

    # the CPU legs run first: their worker processes are forked before this
    # process touches the GPU
    cpu, oracle_c1 = None, None
    if not args.no_cpu_baseline and not args.only and not args.serving_only:
        log("cpu baseline (FP64 oracle, all host cores and one core)...")
        cpu = cpu_baseline()
        log(f"cpu baseline {cpu}")
        oracle_c1 = c1_oracle_newton()
        log(f"oracle C1 Newton step: {oracle_c1['ms']} ms, {oracle_c1['newton_iters']} iterations")
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
    if args.only == "beam":
        print(json.dumps({"beam": beam_bench(symx, torch)}), flush=True)
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
                f"res {rep.residual:.3e}/{rep.residual0:.3e} lin {rep.lin_residual:.2e} "
                f"{rep.ms_total:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = None
        if profile:
            # launches enqueued past PCG convergence only test a flag (< 4 us)
            kt = {"busy": mesh.kernel_times(min_ms=IDLE_MS), "all": mesh.kernel_times()}
            mesh.profile(False)
        return wall * 1e3 / K, reps, kt

    def same_iters(r1, r2):
        return [(a["newton_iters"], a["pcg_iters"]) for a in r1] == \
            [(a["newton_iters"], a["pcg_iters"]) for a in r2]

    def spmv_roofline(ktimes, t_bytes, ms_step, label, bound):
        """Roofline of the SpMV launches of a profiled replay (device times from
        per-launch HIP events; launches past convergence excluded)."""
        busy, allk = ktimes["busy"], ktimes["all"]
        kname = "pcg_spmv"
        launches, total_ms = busy[kname]
        avg_ms = total_ms / max(launches, 1)
        nbytes = algorithmic_bytes(kname, N, nnzb, n_elem, t_bytes)
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        top = max(busy.items(), key=lambda kv: kv[1][1])[0]
        return {"kernel": f"pcg_spmv<{label}>", "bound": bound, "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname, label) if args.n == 64 else None,
                "launches": launches, "avg_ms": round(avg_ms, 5), "algorithmic_bytes": nbytes,
                "idle_launches": allk[kname][0] - launches,
                "share_of_step_time": round(allk[kname][1] / (ms_step * args.steps), 4),
                "dominant_kernel_of_step": top == kname}

    def kernel_table(ktimes, t_bytes):
        busy, allk = ktimes["busy"], ktimes["all"]
        out = {}
        for k, (n, ms) in sorted(allk.items(), key=lambda kv: -kv[1][1]):
            nb_, msb = busy.get(k, (0, 0.0))
            d = {"launches": n, "total_ms": round(ms, 3), "busy_launches": nb_,
                 "busy_avg_ms": round(msb / max(nb_, 1), 5)}
            b_ = algorithmic_bytes(k, N, nnzb, n_elem, t_bytes)
            if b_ and nb_:
                d["busy_gbs"] = round(b_ / (msb / nb_ * 1e-3) / 1e9, 1)
            out[k] = d
        return out

    # FP64 (the paper's precision): timed run without per-kernel events (they
    # add host work to every launch), then a replay of the identical
    # deterministic step sequence with per-kernel start/stop events for the
    # roofline of the dominant kernel
    ms_f64, reps_f64, _ = run_steps(symx.SYMX_F64, args.steps, args.warmup, False)
    log(f"newton f64: {ms_f64:.2f} ms/step")
    ms_f64p, reps_f64p, kt64 = run_steps(symx.SYMX_F64, args.steps, args.warmup, True)
    log(f"newton f64 with kernel events: {ms_f64p:.2f} ms/step")
    roofline = spmv_roofline(kt64, 8, ms_f64, "double", "hbm")
    roofline["timing"] = ("hipExtLaunchKernelGGL start/stop events in a replay of the timed "
                          "steps (identical iteration counts: %s)" % same_iters(reps_f64, reps_f64p))
    log(f"roofline f64 spmv: {roofline}")
    ms_f32r, reps_f32r, kt32 = None, None, None
    roofline32 = None
    if not args.no_f32_newton:
        ms_f32r, reps_f32r, _ = run_steps(symx.SYMX_F32_REFINED, args.steps, args.warmup, False)
        log(f"newton f32_refined: {ms_f32r:.2f} ms/step")
        _, reps_f32p, kt32 = run_steps(symx.SYMX_F32_REFINED, args.steps, args.warmup, True)
        # the float32 matrix and vectors (about 200 MB) fit in the 256 MB
        # Infinity Cache (MALL): its SpMV rate is not an HBM figure
        roofline32 = spmv_roofline(kt32, 4, ms_f32r, "float", "mall")
        roofline32["identical_iteration_counts"] = same_iters(reps_f32r, reps_f32p)
        log(f"roofline f32 spmv (MALL-resident): {roofline32}")
        log(f"kernels f32_refined steps: {kernel_table(kt32, 4)}")
    log(f"kernels f64 steps: {kernel_table(kt64, 8)}")

    extras = {}
    if not args.no_c4:
        extras["c4_precision"] = precision_c4(symx, torch)
        log(f"c4: {extras['c4_precision']}")
    if not args.no_c3:
        extras["c3_mixed"] = mixed_c3(symx, torch)
        log(f"c3: {extras['c3_mixed']}")
    if not args.no_beam:
        extras["beam"] = beam_bench(symx, torch)
    if not args.no_materials:
        extras["materials"] = materials_bench(symx, torch)
    if not args.no_quadratic:
        extras["quadratic_tets"] = high_order_bench(symx, torch, "quadratic")
    if not args.no_cubic:
        extras["cubic_tets"] = high_order_bench(symx, torch, "cubic")
    if not args.no_contacts:
        extras["contacts"] = contact_bench(symx, torch)
    serving = None
    if not args.no_serving:
        log("serving (256 requests, Poisson 200/s)...")
        serving = serving_bench(symx, torch)
        extras["serving"] = serving

    if oracle_c1 is not None:
        c1 = c1_newton_vs_oracle(symx, torch, oracle_c1)
        extras["c1_newton_vs_oracle"] = c1
        log(f"c1 newton step, device vs oracle: {c1}")

    def summary(reps):
        if not reps:
            return None
        lin = [r["lin_residual"] for r in reps if r["lin_residual"] >= 0]
        return {"newton_iters": sum(r["newton_iters"] for r in reps),
                "pcg_iters": sum(r["pcg_iters"] for r in reps),
                "refinements": sum(r["refinements"] for r in reps),
                "dt_halvings": sum(r["dt_halvings"] for r in reps),
                "all_converged": all(r["status"] == 0 for r in reps),
                "max_rel_residual": float("%.3g" % max(r["residual"] / max(r["residual0"], 1e-300)
                                                       for r in reps)),
                "max_lin_residual": float("%.3g" % max(lin)) if lin else None}

    if args.details:
        with open(args.details, "w") as f:
            json.dump({"assembly_kernels_f32": asm_kernels, "kernels_f64_steps": kernel_table(kt64, 8),
                       "kernels_f32_refined_steps": kernel_table(kt32, 4) if kt32 else None,
                       "mesh_setup_s": setup_s, **extras}, f, indent=1)
    ms_pair = {"f64": round(ms_f64, 3),
               "f32_refined": None if ms_f32r is None else round(ms_f32r, 3)}
    # compact summary as the last line of the log (the JSON line follows on stdout)
    log("summary: eval+assembly Melem/s " + ", ".join(f"{k} {v:.0f}" for k, v in melem.items())
        + f"; Newton step ms {ms_pair}; SpMV f64 {roofline['achieved']} GB/s "
        f"(frac {roofline['frac']}), f32 (MALL) "
        f"{None if roofline32 is None else roofline32['achieved']} GB/s; "
        f"cpu oracle {None if cpu is None else cpu['value']} Melem/s on "
        f"{None if cpu is None else cpu['cores']} cores")
    out = {
        "metric": "elem eval+assembly Melem/s, Newton step ms FP32-refined vs FP64; p99 latency",
        "value": round(melem["f64"], 2),
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_f64, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C2 {args.n}^3 cubes x 6 SNH tets: {n_elem} tets, {N} nodes, "
                               f"{nnzb} blocks",
                   "value": "FP64 E+g+BSR-H eval+assembly, no projection",
                   "ms_per_step": "FP64 Newton time step (rtol 1e-6, PCG<=500)"},
        "melem_per_s": {k: round(v, 1) for k, v in melem.items()},
        "newton_step_ms": ms_pair,
        "newton_f64": summary(reps_f64),
        "newton_f32_refined": summary(reps_f32r),
        "p99_latency_ms": None if serving is None else serving["full_budget"]["p99_ms"],
        "serving": None if serving is None else {
            "p50_ms": serving["full_budget"]["p50_ms"], "p99_ms": serving["full_budget"]["p99_ms"],
            "requests_per_s": {k: serving[k]["requests_per_s"]
                               for k in ("full_budget", "saturated", "sequential")},
            "melem_steps_per_s": {k: serving[k]["melem_steps_per_s"]
                                  for k in ("full_budget", "saturated", "sequential")},
            "chunks_per_batch_saturated": serving["saturated"]["chunks_per_batch"]},
        "roofline": roofline,
        "roofline_f32_spmv": roofline32,
        "roofline_assembly": roofline_asm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
