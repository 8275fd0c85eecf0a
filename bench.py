"""Benchmark: element-Jacobi DOF-updates/s and time to a 1e-8 residual drop on one MI355X.

Headline workload (synthetic): steady inviscid flow at Ma 0.001 past the unit sphere (Sec. 4.2
setting) on the equiangular cubed sphere of 6 x 16 x 16 cells x 24 radial shells (36 864
quadratic hexahedra, far field at 20 radii), FR/CPR P = 3 with P-levels {3-2-1-0} and smoothing
counts I{5-10-20-20}, cut-off eps (kappa 1), CFL 30 -> 1e5 by the SER law, blocks rebuilt every 10
V-cycles, started from the free stream and solved to a 1e-8 relative drop of the residual norm.

A step is one whole steady solve (every V-cycle until the 1e-8 drop, with every block rebuild the
schedule asks for): every row of the hot path runs in it. `value` is the DOF-updates per second of
the mixed form (FP32 inverse blocks on the smoother, FP64 residual, update and restriction, the
V-cycles replayed from a HIP graph) over the K timed steps; `ms_per_step` is therefore its time to
the 1e-8 drop. The plain FP64 form (FP64 blocks, eager launches) solves the same problem after it
and both times to 1e-8 are reported. The final stdout line is the compact result; the optional
blocks (`--extra`) go to a side JSON file and to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "element-Jacobi DOF-updates/s + time to 1e-8 residual drop, mixed vs FP64"
P_LEVELS = (3, 2, 1)
N_SMOOTH = (5, 10, 20)
DT = 0.05
SCHEME = 3
HBM_PEAK_GBS = 8000.0


def dof_updates_per_vcycle(ne, p_levels, n_smooth, nv=4, dim=2):
    """sum over levels of (sweeps per V-cycle) * DOF_l: 2 n_l sweeps on every level but the
    coarsest, which smooths n_L times once."""
    tot = 0
    last = len(p_levels) - 1
    for l, (P, n) in enumerate(zip(p_levels, n_smooth)):
        sweeps = n if l == last else 2 * n
        tot += sweeps * ne * nv * (P + 1) ** dim
    return tot


def cpu_baseline(n_cells=2, n_shells=2, plev=(3, 2, 1, 0), nsm=(5, 10, 20, 20)):
    """The CPU oracle on a bounded sample of the headline workload: one block rebuild on every level
    and one V-cycle of the same steady sphere problem (same P-levels, smoothing counts, cut-off eps
    and CFL start) on a cubed sphere of 6 x n_cells^2 x n_shells hexahedra, with the BLAS/LAPACK
    pool limited to the host cores available to this process (at most 16). DOF-updates/s =
    DOF-updates of one V-cycle / (V-cycle time + rebuild time / 10): the rebuild amortised as the
    schedule does (one per 10 V-cycles)."""
    from threadpoolctl import threadpool_limits

    from oracle import gas as OG
    from oracle import solver as OS
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    mesh = W.cubed_sphere_mesh(n_cells, n_shells)
    fs = W.FreeStream3Spec()
    gas = OG.Gas(gamma=fs.gamma, rgas=fs.rgas, eps_mode="cutoff", ma_inf=fs.ma_inf, kappa=1.0)
    with threadpool_limits(threads):
        opts = OS.PMGOptions(p_levels=plev, n_smooth=nsm, use_cfl=True, cfl_init=30.0, cfl_max=1e5,
                             freeze_at_max=False)
        sol = OS.PMGSolver(mesh, gas, opts, q_inf=fs.freestream())
        lev = sol.levels[0]
        q = np.broadcast_to(fs.freestream(), (lev.ne, lev.npts, 5)).copy()
        sol.c_mass, sol.src = 0.0, None
        sol.dtau = opts.cfl_init * sol.dtau_min(q)
        t0 = time.perf_counter()
        sol.build_D(0, q)
        qb = q
        for l in range(1, len(plev)):
            qb = OS.restrict(qb, plev[l - 1], plev[l], 3)
            sol.build_D(l, qb)
        t_build = time.perf_counter() - t0
        sol.refresh_now = False
        t0 = time.perf_counter()
        sol.vcycle(0, q, None)
        t_vc = time.perf_counter() - t0
    per_vc = dof_updates_per_vcycle(mesh.n_elements, plev, nsm, nv=5, dim=3)
    cpu = ""
    try:
        cpu = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        cpu = platform.processor() or platform.machine()
    return {"value": per_vc / (t_vc + t_build / 10.0), "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, sphere P{{{'-'.join(map(str, plev))}}} on {mesh.n_elements} hexahedra "
                       f"(6x{n_cells}x{n_cells}x{n_shells}): rebuild {t_build:.1f} s + one V-cycle {t_vc:.1f} s, "
                       "rebuild amortised 1/10"),
            "cpu": cpu}


FORMS = {"mixed": (32, True), "fp64": (64, False)}   # (block precision, graph replay)
TOLS = (1e-4, 1e-6, 1e-8)


def time_to_tolerances(stage_stats):
    """Per stage: wall time until r_m / r_0 first fell to each tolerance (None if never), from
    the residual history and the stage's mean V-cycle time."""
    out = {f"{t:.0e}": [] for t in TOLS}
    floors = []
    for st in stage_stats:
        h = np.asarray(st["history"])
        floors.append(float(h.min() / h[0]))
        per_vc = st["seconds"] / max(st["n_vcycles"], 1)
        for t in TOLS:
            hit = np.nonzero(h / h[0] <= t)[0]
            out[f"{t:.0e}"].append(float(hit[0] * per_vc) if hit.size else None)
    return out, floors


def run_form(api, torch, levels, q0, form, scheme, dt, steps, warmup, max_vcycles, work, later_guess="predictor",
             lookahead=1):
    """`steps` ESDIRK steps from q0 (after `warmup` untimed ones): the first step's stages start
    from the previous stage value (q0 is not a solved time level), the later ones from
    `later_guess` (the explicit predictor by default)."""
    prec, graph = FORMS[form]
    facs = [api.Factors(lv, prec) for lv in levels]
    solvers = [api.StageSolver(levels, facs, N_SMOOTH if len(levels) == 3 else (5, 10, 20)[:len(levels)],
                               dtau_init=0.01, dtau_max=10.0, ser_exponent=1.5, refresh_every=10,
                               freeze_at_max=True, tol_rel=1e-8, max_vcycles=max_vcycles, use_graph=graph,
                               stage_guess=g, lookahead=lookahead) for g in ("previous", later_guess)]
    q = q0.clone()
    for k in range(warmup):
        api.esdirk_step(solvers[min(k, 1)], scheme, dt, q, work, raise_on_error=False)
    q.copy_(q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stage_stats = []
    for k in range(steps):
        stage_stats += api.esdirk_step(solvers[min(k, 1)], scheme, dt, q, work, raise_on_error=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return facs, solvers[0], q, stage_stats, elapsed


AIRFOIL_HIERARCHIES = (("P4-2-1", (4, 2, 1), (5, 10, 20)), ("P4-3-2-1-0", (4, 3, 2, 1, 0), (5, 10, 20, 20, 20)))


def airfoil_block(api, torch, forms, max_vcycles, kernel_reps):
    """Steady inviscid flow at Ma 0.001, 2 degrees, around the 12% symmetric profile on the
    128 x 64 quadratic O-mesh, P = 4 (Sec. 4.2): for each hierarchy and block precision, one
    steady solve from the free stream with CFL 1e2 -> 1e5 (blocks rebuilt every 10 V-cycles),
    its V-cycle rate, residual history and time to each tolerance, and the live duration of the
    fine-level fused sweep."""
    mesh, fs = W.airfoil_config3()
    qinf = fs.freestream()
    out = {"workload": "NACA-type 12% symmetric profile, O-mesh 128x64 quadratic quads, Ma 0.001, 2 deg, "
                       "slip wall + far field, cut-off eps (kappa 1), steady, CFL 1e2 -> 1e5, "
                       "blocks rebuilt every 10 V-cycles", "elements": mesh.n_elements}
    for name, plev, nsm in AIRFOIL_HIERARCHIES:
        levels = [api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0,
                            q_inf=qinf, q_ref=qinf) for P in plev]
        per_vc = dof_updates_per_vcycle(levels[0].ne, plev, nsm)
        res = {"dof_updates_per_vcycle": per_vc, "n_smooth": list(nsm)}
        for form in forms:
            prec, graph = FORMS[form]
            facs = [api.Factors(lv, prec) for lv in levels]
            kw = dict(tol_rel=1e-8, use_graph=graph, use_cfl=True, cfl_init=1e2, cfl_max=1e5, freeze_at_max=False)
            q = levels[0].new_state()                    # the free stream (zero offset)
            api.StageSolver(levels, facs, nsm, max_vcycles=12, **kw).solve(q, raise_on_error=False)   # warm-up
            q.zero_()
            solver = api.StageSolver(levels, facs, nsm, max_vcycles=max_vcycles, **kw)
            torch.cuda.synchronize()
            st = solver.solve(q, raise_on_error=False)
            h = np.asarray(st["history"]) / st["history"][0]
            per = st["seconds"] / max(st["n_vcycles"], 1)
            ttt = {}
            for t in TOLS:
                hit = np.nonzero(h <= t)[0]
                ttt[f"{t:.0e}"] = float(hit[0] * per) if hit.size else None
            fin = np.isfinite(h)
            # live duration of the fine-level fused residual + sweep (alpha_r = 0 keeps q fixed)
            qk = q.clone()
            api.ejacobi_sweep(levels[0], facs[0], qk, 2, alpha_r=0.0)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            api.ejacobi_sweep(levels[0], facs[0], qk, kernel_reps, alpha_r=0.0)
            ev1.record()
            torch.cuda.synchronize()
            k_ms = ev0.elapsed_time(ev1) / kernel_reps
            n = levels[0].n
            bpd = (4 if prec == 32 else 8) * n + 24
            kbytes = levels[0].ne * n * bpd
            res[form] = {"status": st["status"], "vcycles": st["n_vcycles"], "block_rebuilds": st["n_refresh"],
                         "seconds": st["seconds"], "ms_per_vcycle": 1e3 * per,
                         "dof_updates_per_s": per_vc * st["n_vcycles"] / st["seconds"],
                         "time_to_tol_s": ttt, "min_rel_residual": float(np.min(h[fin])),
                         "final_rel_residual": float(h[fin][-1]), "dtau_min": st["dtau_min"],
                         "history_every_25": [float(x) for x in h[::25]],
                         "fine_sweep_kernel_ms": k_ms, "fine_sweep_bytes_per_launch": kbytes,
                         "fine_sweep_hbm_frac": kbytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "fine_sweep_traffic": measured_traffic(PROFILE_PMC_AIRFOIL) if prec == 32 else None}
            del facs, solver
        out[name] = res
    return out


def airfoil_lines_block(api, torch, max_vcycles, kernel_reps, plev=(4, 2, 1), nsm=(5, 10, 20)):
    """The same steady airfoil solve with FP32 blocks and graph replay, smoothed by element Jacobi
    and by element-line Jacobi along the O-mesh's radial lines (128 lines of 64 elements, the
    direction in which the cells are stretched) on every level: V-cycles, time to each tolerance,
    and the live duration of the fine-level line sweep (residual + forward and backward block
    substitution) against its algorithmic bytes."""
    mesh, fs = W.airfoil_config3()
    qinf = fs.freestream()
    nw, nr = 128, 64                                     # element e = i + 128 j (i round, j outwards)
    radial = np.arange(nw)[:, None] + nw * np.arange(nr)[None, :]
    levels = [api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0,
                        q_inf=qinf, q_ref=qinf) for P in plev]
    per_vc = dof_updates_per_vcycle(levels[0].ne, plev, nsm)
    out = {"workload": f"airfoil O-mesh {nw}x{nr}, P{{{'-'.join(map(str, plev))}}} I{{{'-'.join(map(str, nsm))}}}, "
                       "FP32 blocks, graph replay, steady, CFL 1e2 -> 1e5",
           "lines": f"{nw} radial lines of {nr} elements", "dof_updates_per_vcycle": per_vc}
    kw = dict(tol_rel=1e-8, use_graph=True, use_cfl=True, cfl_init=1e2, cfl_max=1e5, freeze_at_max=False)
    for smoother in ("element", "line"):
        if smoother == "line":
            facs = [api.LineFactors(lv, radial, 32) for lv in levels]
        else:
            facs = [api.Factors(lv, 32) for lv in levels]
        q = levels[0].new_state()
        api.StageSolver(levels, facs, nsm, max_vcycles=12, **kw).solve(q, raise_on_error=False)   # warm-up
        q.zero_()
        solver = api.StageSolver(levels, facs, nsm, max_vcycles=max_vcycles, **kw)
        torch.cuda.synchronize()
        st = solver.solve(q, raise_on_error=False)
        h = np.asarray(st["history"]) / st["history"][0]
        per = st["seconds"] / max(st["n_vcycles"], 1)
        ttt = {}
        for t in TOLS:
            hit = np.nonzero(h <= t)[0]
            ttt[f"{t:.0e}"] = float(hit[0] * per) if hit.size else None
        fin = np.isfinite(h)
        qk = q.clone()
        api.ejacobi_sweep(levels[0], facs[0], qk, 2, alpha_r=0.0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        api.ejacobi_sweep(levels[0], facs[0], qk, kernel_reps, alpha_r=0.0)
        ev1.record()
        torch.cuda.synchronize()
        k_ms = ev0.elapsed_time(ev1) / kernel_reps
        n = levels[0].n
        # element: one pass over the FP32 inverses + 24 B/DOF of state; line: the inverses once and
        # C_k, B_k (4(P+1) FP32 columns each) once, 24 B/DOF for the residual kernel and 56 B/DOF
        # for the substitutions' right-hand side, intermediates and state
        nj = 4 * (plev[0] + 1)
        bpd = 4 * n + 24 if smoother == "element" else 4 * n + 8 * nj + 80
        kbytes = levels[0].ne * n * bpd
        out[smoother] = {"status": st["status"], "vcycles": st["n_vcycles"], "block_rebuilds": st["n_refresh"],
                         "seconds": st["seconds"], "ms_per_vcycle": 1e3 * per,
                         "dof_updates_per_s": per_vc * st["n_vcycles"] / st["seconds"],
                         "time_to_tol_s": ttt, "min_rel_residual": float(np.min(h[fin])),
                         "final_rel_residual": float(h[fin][-1]),
                         "history_every_25": [float(x) for x in h[::25]],
                         "fine_sweep_ms": k_ms, "fine_sweep_bytes": kbytes,
                         "fine_sweep_hbm_frac": kbytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del facs, solver
    return out


def sphere_block(api, torch, forms, max_vcycles, kernel_reps, plev=(2, 1, 0), nsm=(5, 10, 20),
                 profile_pmc=None, cfl_init=1e2):
    """Steady inviscid flow at Ma 0.001 past the unit sphere on the 6 x 16 x 16 x 24 cubed sphere of
    27-node hexahedra (36 864 elements), P{2-1-0} (135 x 135 element blocks) or P{3-2-1-0} (320 x
    320): for each block precision one steady solve from the free stream with CFL cfl_init -> 1e5
    (blocks rebuilt every 10 V-cycles), its V-cycle rate, residual history, time to each
    tolerance, and the live durations of the fine-level fused sweep and block rebuild. From the
    impulsive start P{3-2-1-0} diverges at CFL_init 1e2 on this mesh and takes 30."""
    profile_pmc = profile_pmc or PROFILE_PMC_SPHERE
    mesh, fs = W.sphere_config5()
    qinf = fs.freestream()
    levels = [api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0,
                        q_inf=qinf, q_ref=qinf) for P in plev]
    per_vc = dof_updates_per_vcycle(levels[0].ne, plev, nsm, nv=5, dim=3)
    hier = "P{" + "-".join(str(P) for P in plev) + "}"
    out = {"workload": "unit sphere, cubed sphere 6x16x16 cells x 24 shells (36864 quadratic hexahedra, far "
                       "field at r = 20), Ma 0.001, slip wall + far field, cut-off eps (kappa 1), steady, "
                       f"{hier}, CFL 1e2 -> 1e5, blocks rebuilt every 10 V-cycles",
           "elements": mesh.n_elements, "block_size": levels[0].n, "dof_updates_per_vcycle": per_vc,
           "n_smooth": list(nsm)}
    for form in forms:
        prec, graph = FORMS[form]
        tuned = [lv.autotune(precision=prec, reps=5) for lv in levels]   # setup, before the solve
        facs = [api.Factors(lv, prec) for lv in levels]
        kw = dict(tol_rel=1e-8, use_graph=graph, use_cfl=True, cfl_init=cfl_init, cfl_max=1e5, freeze_at_max=False)
        q = levels[0].new_state()
        api.StageSolver(levels, facs, nsm, max_vcycles=12, **kw).solve(q, raise_on_error=False)   # warm-up
        q.zero_()
        solver = api.StageSolver(levels, facs, nsm, max_vcycles=max_vcycles, **kw)
        torch.cuda.synchronize()
        st = solver.solve(q, raise_on_error=False)
        h = np.asarray(st["history"]) / st["history"][0]
        per = st["seconds"] / max(st["n_vcycles"], 1)
        ttt = {}
        for t in TOLS:
            hit = np.nonzero(h <= t)[0]
            ttt[f"{t:.0e}"] = float(hit[0] * per) if hit.size else None
        fin = np.isfinite(h)
        qk = q.clone()
        api.ejacobi_sweep(levels[0], facs[0], qk, 2, alpha_r=0.0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        api.ejacobi_sweep(levels[0], facs[0], qk, kernel_reps, alpha_r=0.0)
        ev1.record()
        torch.cuda.synchronize()
        k_ms = ev0.elapsed_time(ev1) / kernel_reps
        ev0.record()
        api.fr_element_jacobian(levels[0], q, st["dtau_min"] * 1e2, 0.0, facs[0])
        ev1.record()
        torch.cuda.synchronize()
        jac_ms = ev0.elapsed_time(ev1)
        n = levels[0].n
        npad = (n + 3) // 4 * 4             # block rows are stored padded to a multiple of 4
        kbytes = levels[0].ne * n * ((4 if prec == 32 else 8) * npad + 24)
        out[form] = {"status": st["status"], "vcycles": st["n_vcycles"], "block_rebuilds": st["n_refresh"],
                     "seconds": st["seconds"], "ms_per_vcycle": 1e3 * per,
                     "dof_updates_per_s": per_vc * st["n_vcycles"] / st["seconds"],
                     "time_to_tol_s": ttt, "min_rel_residual": float(np.min(h[fin])) if fin.any() else None,
                     "final_rel_residual": float(h[fin][-1]) if fin.any() else None, "dtau_min": st["dtau_min"],
                     "history_every_25": [float(x) for x in h[::25]],
                     "fine_sweep_kernel_ms": k_ms, "fine_sweep_bytes_per_launch": kbytes,
                     "fine_sweep_hbm_frac": kbytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     # the counters were taken with the default grouping of the fine level
                     "fine_sweep_traffic": (measured_traffic(profile_pmc, KERNEL_SOURCES_3D)
                                            if prec == 32 and levels[0].epw()[0] == levels[0].epw()[1][0]
                                            else None),
                     "elements_per_workgroup": [lv.epw()[0] for lv in levels],
                     "autotune_us_per_residual_and_sweep": [{str(k): v for k, v in
                                                             t["us_per_residual_and_sweep"].items()} for t in tuned],
                     "fine_block_rebuild_ms": jac_ms,
                     "fine_block_rebuild_gj_tflops": levels[0].ne * 2.0 * n ** 3 / (jac_ms * 1e-3) / 1e12}
        del facs, solver
    return out


def newton_krylov_block(api, torch, levels, q0, forms):
    """The first implicit ESDIRK3 stage of the 64x64 vortex solved to a 1e-8 drop two ways: the FAS
    pseudo-transient solve of the main measurement (dtau 0.01 -> 10, at most 400 V-cycles) and the
    Newton-Krylov solve with that V-cycle as preconditioner of flexible GMRES (10 directions per
    Newton step, GMRES tolerance 0.05, dtau 10 -> 1e4, finite-difference scales 1e-3); then one
    whole ESDIRK3 step of the main measurement with every stage solved by Newton-Krylov."""
    g = 1767732205903.0 / 4055673282236.0
    L0 = levels[0]
    qc = torch.empty_like(q0)
    api.fr_conservative(L0, q0, qc)
    R1 = torch.empty_like(q0)
    api.fr_residual(L0, q0, R1)
    stage = dict(omega=g, dt=DT, qc_n=qc, R_prev=[R1], a_row=[g])
    out = {"workload": "first implicit ESDIRK3 stage (dt 0.05) of the 64x64 jittered vortex, P{3-2-1}, "
                       "I{5-10-20}, stop at r/r0 <= 1e-8"}
    for form in forms:
        prec, graph = FORMS[form]
        facs = [api.Factors(lv, prec) for lv in levels]
        res = {}
        for name, dtau, nk in (("fas", (0.01, 10.0), None), ("newton_krylov", (10.0, 1e4), True)):
            solver = api.StageSolver(levels, facs, N_SMOOTH, dtau_init=dtau[0], dtau_max=dtau[1], tol_rel=1e-8,
                                     max_vcycles=400, use_graph=graph)
            for rep in range(2):                              # the first run captures the graph
                q = q0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if nk:
                    st = api.nk_stage_solve(solver, q, krylov_dim=10, eta=0.05, max_newton=60, raise_on_error=False,
                                            **stage)
                else:
                    st = solver.solve(q, raise_on_error=False, **stage)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
            h = np.asarray(st["history"]) / st["history"][0]
            res[name] = {"status": st["status"], "seconds": el, "final_rel_residual": float(h[-1]),
                         "vcycles": st["n_krylov"] if nk else st["n_vcycles"], "dtau_range": list(dtau)}
            if nk:
                res[name]["newton_steps"] = st["n_newton"]
        # one whole ESDIRK3 step, every implicit stage solved by Newton-Krylov to the 1e-8 drop
        Ab = api.esdirk_butcher(SCHEME)
        solver = api.StageSolver(levels, facs, N_SMOOTH, dtau_init=10.0, dtau_max=1e4, tol_rel=1e-8, max_vcycles=400,
                                 use_graph=graph)
        q = q0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qcn = torch.empty_like(q0)
        api.fr_conservative(L0, q, qcn)
        Rs = [torch.empty_like(q0)]
        api.fr_residual(L0, q, Rs[0])
        per_stage = []
        for i in range(1, Ab.shape[0]):
            st = api.nk_stage_solve(solver, q, krylov_dim=10, eta=0.05, max_newton=120, omega=Ab[1, 1], dt=DT,
                                    qc_n=qcn, R_prev=Rs, a_row=list(Ab[i, :i]), raise_on_error=False)
            per_stage.append(st)
            if i < Ab.shape[0] - 1:
                Rs.append(torch.empty_like(q0))
                api.fr_residual(L0, q, Rs[-1])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res["newton_krylov_esdirk3_step"] = {
            "seconds": el, "stages_converged_to_1e-8": sum(st["status"] == 0 for st in per_stage),
            "stages": len(per_stage), "newton_steps": [st["n_newton"] for st in per_stage],
            "directions": [st["n_krylov"] for st in per_stage],
            "final_rel_residual": [st["history"][-1] / st["history"][0] for st in per_stage]}
        out[form] = res
        del facs
    return out


def viscous_batch_block(api, torch, vcycles_per_stage, steps=1):
    """Eight independent viscous cases (Re 5000, Ma 0.001, no-slip adiabatic wall, 256 x 96
    O-mesh, seeded incidence and P in {2, 3, 4}), one ESDIRK3 step of dt = 0.05 from a free stream
    ramped to zero at the wall, every stage run for a fixed budget of V-cycles (CFL 1 -> 1e2).
    Three forms on the same work: all cases as one batch with FP32 blocks and graph replay; the
    same cases one after another with FP32 blocks and graph replay (the effect of batching alone);
    and one after another with FP64 blocks (eager)."""
    mesh, cases = W.viscous_config4()
    nsm_of = {4: (5, 10, 20, 20), 3: (5, 10, 20), 2: (5, 10, 20)}
    stages = api.esdirk_stages(3)
    dt = 0.05
    starts, per_vc = [], []
    sample_levels = {}
    for c in cases:
        if c.P not in sample_levels:
            sample_levels[c.P] = api.Level(mesh, c.P, q_inf=c.spec.freestream())
        xy = np.moveaxis(sample_levels[c.P].points(), 0, -1)
        starts.append(W.viscous_start_state(c.spec, xy) - c.spec.freestream())
        per_vc.append(dof_updates_per_vcycle(mesh.n_elements, c.p_levels, nsm_of[c.P]))
    del sample_levels

    def solvers_for(prec, graph):
        out = []
        for c in cases:
            qinf = c.spec.freestream()
            levels = [api.Level(mesh, P, gamma=c.spec.gamma, rgas=c.spec.rgas, eps_mode=1, ma_inf=c.spec.ma_inf,
                                kappa=1.0, q_inf=qinf, q_ref=qinf, mu=c.mu, prandtl=c.prandtl) for P in c.p_levels]
            facs = [api.Factors(lv, prec) for lv in levels]
            out.append(api.StageSolver(levels, facs, nsm_of[c.P], use_graph=graph, use_cfl=True, cfl_init=1.0,
                                       cfl_max=1e2, freeze_at_max=False, tol_rel=1e-30,
                                       max_vcycles=vcycles_per_stage))
        return out

    res = {"workload": "8 viscous cases, Re 5000, Ma 0.001, no-slip adiabatic wall, O-mesh 256x96 "
                       "(24576 elements), incidence U[0,6] deg and P in {2,3,4} from default_rng(5000), "
                       "ESDIRK3 dt 0.05 from a wall-ramped free stream, CFL 1 -> 1e2, "
                       f"{vcycles_per_stage} V-cycles per stage",
           "cases": [{"alpha_deg": c.alpha_deg, "P": c.P, "p_levels": list(c.p_levels)} for c in cases]}
    for form, (prec, graph, batched) in (("mixed_batched", (32, True, True)), ("mixed_sequential", (32, True, False)),
                                         ("fp64_sequential", (64, False, False))):
        solvers = solvers_for(prec, graph)
        qs = [torch.from_numpy(np.ascontiguousarray(np.moveaxis(q0, -1, 0))).cuda() for q0 in starts]
        works = [torch.zeros((stages,) + sv.levels[0].shape, dtype=torch.float64, device="cuda") for sv in solvers]
        batch = api.Batch(solvers) if batched else None

        def one_step(qq):
            if batched:
                return batch.esdirk_step(3, [dt] * len(cases), qq, works, raise_on_error=False)
            return [api.esdirk_step(sv, 3, dt, q, w, raise_on_error=False) for sv, q, w in zip(solvers, qq, works)]

        one_step([q.clone() for q in qs])                      # warm-up (graph capture, first touch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = []
        for _ in range(steps):
            st = one_step(qs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        upd = sum(per_vc[c] * sum(x["n_vcycles"] for x in st[c]) for c in range(len(cases))) * steps
        res[form] = {"elapsed_s": el, "dof_updates_per_s": upd / el, "dof_updates": upd,
                     "stage_status": [[x["status"] for x in st[c]] for c in range(len(cases))],
                     "stage_vcycles": [[x["n_vcycles"] for x in st[c]] for c in range(len(cases))],
                     "stage_rel_residual": [[(x["history"][-1] / x["history"][0]) if x["history"] and x["history"][0]
                                             else None for x in st[c]] for c in range(len(cases))]}
        if batch is not None:
            batch.close()
        del solvers, works, qs
        torch.cuda.empty_cache()
    if res["fp64_sequential"]["elapsed_s"] > 0:
        res["speedup_mixed_batched_over_fp64_sequential"] = (res["fp64_sequential"]["elapsed_s"]
                                                             / res["mixed_batched"]["elapsed_s"])
        res["speedup_batching_alone"] = res["mixed_sequential"]["elapsed_s"] / res["mixed_batched"]["elapsed_s"]
    return res


PROFILE_PMC = os.path.join(ROOT, "profiles", "k_fr_sweep_vortex64_P321_pmc.txt")
PROFILE_PMC_AIRFOIL = os.path.join(ROOT, "profiles", "k_fr_sweep_airfoil128x64_P4_pmc.txt")
PROFILE_PMC_SPHERE = os.path.join(ROOT, "profiles", "k_fr3_sweep_sphere16x16x24_P2_pmc.txt")
PROFILE_PMC_SPHERE3 = os.path.join(ROOT, "profiles", "k_fr3_sweep_sphere16x16x24_P3_pmc.txt")


KERNEL_SOURCES_2D = ("fr_kernels.hip", "physics.hpp", "internal.hpp", "block_loads.hpp", "vcycle.hpp")
KERNEL_SOURCES_3D = ("fr3_kernels.hip", "hex_points.hpp", "physics3.hpp", "physics.hpp", "internal.hpp", "block_loads.hpp")


def kernel_source_hash(files=KERNEL_SOURCES_2D):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1908_03972_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=PROFILE_PMC, files=KERNEL_SOURCES_2D):
    """HBM bytes per launch of the dominant fused sweep from a committed counter summary, or None
    when the kernel sources have changed since the counters were taken."""
    try:
        vals = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                    if line.startswith(("traffic_bytes_per_launch:", "kernel_source_hash:")))
    except (OSError, ValueError):
        return None
    if vals.get("kernel_source_hash", "").strip() != kernel_source_hash(files):
        return None
    return float(vals["traffic_bytes_per_launch"])


_T0 = time.perf_counter()


def progress(what):
    """One line on stderr per finished block of the run (the JSON line goes to stdout)."""
    print(f"bench: {what} done at {time.perf_counter() - _T0:.1f} s", file=sys.stderr, flush=True)


def vortex_block(api, torch, forms, steps, warmup, max_vcycles, kernel_reps, autotune=True):
    """Config 2: isentropic vortex (Ma 0.005) on the periodic 64 x 64 jittered quad mesh, P{3-2-1},
    I{5-10-20}, ESDIRK3 steps of dt 0.05 from the analytic vortex, every stage to 1e-8 or
    max_vcycles, in both forms; the fine level's FP32 inverses (67 MB) fit the 256 MB Infinity
    Cache, so its sweep fraction is not an HBM figure."""
    mesh, vs = W.vortex_config2()
    qinf = vs.freestream()
    levels = [api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf, q_inf=qinf, q_ref=qinf)
              for P in P_LEVELS]
    xy = levels[0].points()
    q0 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(vs.state(xy[0], xy[1]) - qinf, -1, 0))).cuda()
    L0 = levels[0]
    work = torch.zeros((api.esdirk_stages(SCHEME),) + L0.shape, dtype=torch.float64, device="cuda")
    per_vc = dof_updates_per_vcycle(L0.ne, P_LEVELS, N_SMOOTH)
    out = {"workload": "isentropic vortex Ma 0.005, periodic 64x64 jittered quads, P{3-2-1} I{5-10-20}, "
                       f"ESDIRK3 dt 0.05, {steps} steps, stages to 1e-8 or {max_vcycles} V-cycles"}
    finals = {}
    for form in forms:
        if autotune:
            for lv in levels:
                lv.autotune(precision=FORMS[form][0], reps=20)
        facs, solver, q, stage_stats, elapsed = run_form(api, torch, levels, q0, form, SCHEME, DT, steps, warmup,
                                                         max_vcycles, work)
        nvc = sum(st["n_vcycles"] for st in stage_stats)
        ttt, floors = time_to_tolerances(stage_stats)
        qk = q.clone()
        c_mass = 1.0 / (DT * 1767732205903.0 / 4055673282236.0)
        api.ejacobi_sweep(L0, facs[0], qk, 2, c_mass=c_mass, alpha_r=0.0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        api.ejacobi_sweep(L0, facs[0], qk, kernel_reps, c_mass=c_mass, alpha_r=0.0)
        ev1.record()
        torch.cuda.synchronize()
        k_ms = ev0.elapsed_time(ev1) / kernel_reps
        prec = FORMS[form][0]
        launch_bytes = L0.ne * L0.n * ((4 if prec == 32 else 8) * L0.n + 24)
        out[form] = {"dof_updates_per_s": nvc * per_vc / elapsed, "ms_per_vcycle": 1e3 * elapsed / max(nvc, 1),
                     "vcycles_per_stage": [st["n_vcycles"] for st in stage_stats],
                     "stages_converged_to_1e-8": sum(st["status"] == 0 for st in stage_stats),
                     "time_to_tol_s_per_stage": ttt, "min_rel_residual_per_stage": floors,
                     "fine_sweep_ms": k_ms, "fine_sweep_bytes": launch_bytes,
                     "fine_sweep_frac_of_8TBs": launch_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "elements_per_workgroup": [lv.epw()[0] for lv in levels]}
        finals[form] = q.detach().cpu().numpy()
        del facs, solver
        if form == "mixed":   # the same steps with one V-cycle per host stopping test
            facs, solver, q, st_off, el_off = run_form(api, torch, levels, q0, form, SCHEME, DT, steps, warmup,
                                                       max_vcycles, work, lookahead=0)
            out[form]["lookahead_off"] = {
                "ms_per_vcycle": 1e3 * el_off / max(sum(st["n_vcycles"] for st in st_off), 1),
                "speedup_of_lookahead": el_off / elapsed,
                "identical_result": bool(np.array_equal(q.detach().cpu().numpy(), finals[form])) and
                [st["history"] for st in st_off] == [st["history"] for st in stage_stats]}
            del facs, solver
    if "mixed" in finals and "fp64" in finals:
        d = finals["fp64"]
        out["mixed_vs_fp64_rel_err"] = (np.linalg.norm((finals["mixed"] - d).reshape(4, -1), axis=1)
                                        / np.linalg.norm(d.reshape(4, -1), axis=1)).tolist()
    return out, levels, q0


def small_vortex_block(api, torch, forms):
    """Config 1: the 8x8 P{2-1-0} ESDIRK2 vortex, five steps, stages to 1e-8 (at most 2000 V-cycles),
    every stage from the previous stage value (on this mesh it takes more stages to 1e-8 than the
    explicit predictor does: 6 of 10 against 4 of 10)."""
    m1, v1 = W.vortex_config1()
    qinf = v1.freestream()
    lv1 = [api.Level(m1, P, gamma=v1.gamma, rgas=v1.rgas, eps_mode=0, ma_inf=v1.ma_inf, q_inf=qinf, q_ref=qinf)
           for P in (2, 1, 0)]
    xy = lv1[0].points()
    q1 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(v1.state(xy[0], xy[1]) - qinf, -1, 0))).cuda()
    w1 = torch.zeros((api.esdirk_stages(2),) + lv1[0].shape, dtype=torch.float64, device="cuda")
    small = {}
    for form in forms:
        _, _, _, sst, el = run_form(api, torch, lv1, q1, form, 2, DT, 5, 1, 2000, w1, later_guess="previous")
        small[form] = {"elapsed_s": el, "stages": len(sst),
                       "stages_converged_to_1e-8": sum(s["status"] == 0 for s in sst),
                       "vcycles_per_stage": [s["n_vcycles"] for s in sst],
                       "time_to_1e-8_s_total": float(sum(s["seconds"] for s in sst))}
    if "mixed" in small and "fp64" in small and small["mixed"]["time_to_1e-8_s_total"] > 0:
        small["speedup_time_to_1e-8_mixed_over_fp64"] = (small["fp64"]["time_to_1e-8_s_total"]
                                                         / small["mixed"]["time_to_1e-8_s_total"])
    return small


TIMEREF_STEPS = {2: (100, 200, 400), 3: (100, 200, 400), 4: (40, 80, 120)}


def time_refinement_block(api, torch, schemes=(2, 3, 4), n=50, prec=32, first_guess="previous", steps=None,
                          later_guess="predictor", ser_floor=False):
    """Sec. 4.1's time-refinement study (Table 1's setting): the isentropic vortex at Ma 0.005 on
    the periodic [-10, 10]^2 square with n x n elements, P5 with P{5-3-1} and I{20-20-40}, dtau
    0.01 -> 10, blocks rebuilt every 10 V-cycles, every implicit stage solved to a 1e-4 relative
    drop (at most 200 V-cycles), advanced over one period t = 20 with the step counts of Table 1,
    the first step's stages from the previous stage value and later ones from the explicit
    predictor (or, with later_guess="previous", from the previous stage value throughout; with
    ser_floor the SER law never takes dtau below 0.01). Errors are RMS over the solution points (uniform mesh) against the exact vortex,
    which is back at its start after one period; orders from successive step sizes, both
    against the exact solution and from the differences of successive solutions."""
    vs = W.VortexSpec(length=20.0, ma_inf=0.005)
    mesh = W.periodic_quad_mesh(n, 20.0)
    qinf = vs.freestream()
    plev, nsm = (5, 3, 1), (20, 20, 40)
    levels = [api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf, q_inf=qinf, q_ref=qinf)
              for P in plev]
    xy = levels[0].points()
    exact = vs.state(xy[0], xy[1])                                     # [Np][Ne][4]
    q0 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(exact - qinf, -1, 0))).cuda()
    facs = [api.Factors(lv, prec) for lv in levels]
    solvers = [api.StageSolver(levels, facs, nsm, dtau_init=0.01, dtau_max=10.0, refresh_every=10, freeze_at_max=True,
                               tol_rel=1e-4, max_vcycles=200, use_graph=True, stage_guess=g, ser_floor=ser_floor)
               for g in (first_guess, later_guess)]

    def rho_u_p(x):
        p, u, T = x[..., 0], x[..., 1], x[..., 3]
        return np.stack([p / (vs.rgas * T), u, p], axis=-1)

    ref = rho_u_p(exact)
    out = {"workload": f"vortex Ma 0.005, periodic [-10,10]^2, {n}x{n} quads, P5, P{{5-3-1}} I{{20-20-40}}, "
                       f"dtau 0.01->10, stage tol 1e-4, one period t=20, FP{prec} blocks",
           "error": "RMS over solution points against the exact vortex (rho, u, p)",
           "stage_guess": [first_guess, later_guess], "ser_floor": bool(ser_floor)}
    for scheme in schemes:
        res = {"dt": [], "err": [], "stages": 0, "stages_converged": 0, "vcycles": 0, "seconds": 0.0}
        sols = []
        for nsteps in (steps or TIMEREF_STEPS)[scheme]:
            dt = 20.0 / nsteps
            q = q0.clone()
            work = torch.zeros((api.esdirk_stages(scheme),) + levels[0].shape, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(nsteps):
                st = api.esdirk_step(solvers[min(k, 1)], scheme, dt, q, work, raise_on_error=False)
                res["stages"] += len(st)
                res["stages_converged"] += sum(x["status"] == 0 for x in st)
                res["vcycles"] += sum(x["n_vcycles"] for x in st)
                bad = [x["status"] for x in st if x["status"] not in (0, -6)]
                if k % 25 == 0 or bad:
                    print(f"bench: ESDIRK{scheme} t/{nsteps} step {k}: statuses {[x['status'] for x in st]} "
                          f"V-cycles {[x['n_vcycles'] for x in st]} "
                          f"r/r0 {[x['history'][-1] / x['history'][0] for x in st if x['history'] and x['history'][0]]}",
                          file=sys.stderr, flush=True)
                if bad:
                    res["failed_at_step"] = k
                    break
            torch.cuda.synchronize()
            res["seconds"] += time.perf_counter() - t0
            qh = np.moveaxis(q.cpu().numpy(), 0, -1) + qinf
            sols.append(rho_u_p(qh))
            res["dt"].append(dt)
            res["err"].append(np.sqrt(np.mean((sols[-1] - ref).reshape(-1, 3) ** 2, axis=0)).tolist())
            progress(f"time refinement ESDIRK{scheme} dt = t/{nsteps}")
        e = np.array(res["err"])
        r = np.array((steps or TIMEREF_STEPS)[scheme], float)
        res["order_vs_exact"] = (np.log(e[:-1] / e[1:]) / np.log(r[1:, None] / r[:-1, None])).tolist()
        if len(sols) == 3:
            d1 = np.sqrt(np.mean((sols[1] - sols[0]).reshape(-1, 3) ** 2, axis=0))
            d2 = np.sqrt(np.mean((sols[2] - sols[1]).reshape(-1, 3) ** 2, axis=0))
            if r[1] / r[0] == r[2] / r[1]:                        # equal ratios: the classic estimate
                res["order_self"] = (np.log(d1 / d2) / np.log(r[1] / r[0])).tolist()
        out[f"esdirk{scheme}"] = res
    return out


HEAD_PLEV = (3, 2, 1, 0)
HEAD_NSM = (5, 10, 20, 20)
HEAD_CFL = (30.0, 1e5)


def sphere_headline(api, torch, steps, warmup, fp64_solves, max_vcycles, kernel_reps, autotune=True):
    """The headline: K timed steady solves of the sphere at P{3-2-1-0} in the mixed form, then the
    plain FP64 form on the same problem, the live duration of the fine-level fused sweep (the
    dominant kernel) and of the fine-level block rebuild."""
    mesh, fs = W.sphere_config5()
    qinf = fs.freestream()
    levels = [api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0,
                        q_inf=qinf, q_ref=qinf) for P in HEAD_PLEV]
    L0 = levels[0]
    per_vc = dof_updates_per_vcycle(L0.ne, HEAD_PLEV, HEAD_NSM, nv=5, dim=3)
    res = {"elements": L0.ne, "dof_fine": L0.ne * L0.n, "dof_updates_per_vcycle": per_vc}
    finals = {}
    for form, nsolve, nwarm in (("mixed", steps, warmup), ("fp64", fp64_solves, 1)):
        if nsolve <= 0:
            continue
        prec, graph = FORMS[form]
        if autotune:
            for lv in levels:
                lv.autotune(precision=prec, reps=5)             # setup, outside the timed region
        facs = [api.Factors(lv, prec) for lv in levels]
        solver = api.StageSolver(levels, facs, HEAD_NSM, tol_rel=1e-8, use_graph=graph, use_cfl=True,
                                 cfl_init=HEAD_CFL[0], cfl_max=HEAD_CFL[1], freeze_at_max=False,
                                 max_vcycles=max_vcycles)
        q = L0.new_state()
        for _ in range(nwarm):
            q.zero_()                                            # the free stream (zero offset)
            solver.solve(q, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = []
        for _ in range(nsolve):
            q.zero_()
            sts.append(solver.solve(q, raise_on_error=False))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        nvc = sum(st["n_vcycles"] for st in sts)
        r = {"solves": nsolve, "elapsed_s": elapsed, "ms_per_solve": 1e3 * elapsed / nsolve,
             "dof_updates_per_s": per_vc * nvc / elapsed, "vcycles": [st["n_vcycles"] for st in sts],
             "rebuilds": [st["n_refresh"] for st in sts], "status": [st["status"] for st in sts],
             "final_rel_residual": [st["history"][-1] / st["history"][0] for st in sts],
             "ms_per_vcycle": 1e3 * elapsed / max(nvc, 1), "elements_per_workgroup": [lv.epw()[0] for lv in levels]}
        # live per-launch duration of the dominant kernel, the fine-level fused residual + sweep,
        # timed with HIP events on the stream the library launches on (torch's current stream);
        # alpha_r = 0 keeps the converged state fixed, the kernel does the same work
        qk = q.clone()
        api.ejacobi_sweep(L0, facs[0], qk, 2, alpha_r=0.0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        api.ejacobi_sweep(L0, facs[0], qk, kernel_reps, alpha_r=0.0)
        ev1.record()
        torch.cuda.synchronize()
        r["sweep_ms"] = ev0.elapsed_time(ev1) / kernel_reps
        r["sweep_bytes"] = L0.ne * L0.n * ((4 if prec == 32 else 8) * L0.n + 24)
        ev0.record()
        api.fr_element_jacobian(L0, q, 1e2 * api.dtau_min(L0, q), 0.0, facs[0])
        ev1.record()
        torch.cuda.synchronize()
        r["rebuild_ms"] = ev0.elapsed_time(ev1)
        finals[form] = q.detach().cpu().numpy()
        res[form] = r
        del facs, solver
        torch.cuda.empty_cache()
        progress(f"sphere P{{3-2-1-0}} {form}: {nsolve} solves, {r['ms_per_solve']:.0f} ms each")
    if "mixed" in finals and "fp64" in finals:
        d = finals["fp64"]
        res["mixed_vs_fp64_rel_err"] = (np.linalg.norm((finals["mixed"] - d).reshape(5, -1), axis=1)
                                        / np.linalg.norm(d.reshape(5, -1), axis=1)).tolist()
    return res


EXTRAS = ("vortex", "small", "nk", "airfoil", "lines", "viscous", "sphere2", "timeref")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steady solves of the headline (mixed form)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-solves", type=int, default=2, help="timed solves of the plain FP64 form")
    ap.add_argument("--max-vcycles", type=int, default=200)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default elements per workgroup")
    ap.add_argument("--extra", default="", help=f"comma list of further blocks: {','.join(EXTRAS)} or all")
    ap.add_argument("--only-extra", action="store_true",
                    help="run only the --extra blocks (no headline, no JSON bench line): for profiling them")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="side file for the full results (the extra blocks, per-solve lists)")
    ap.add_argument("--vortex-vcycles", type=int, default=400)
    ap.add_argument("--airfoil-vcycles", type=int, default=600)
    ap.add_argument("--sphere-vcycles", type=int, default=200)
    ap.add_argument("--viscous-vcycles", type=int, default=10, help="V-cycles per stage in the viscous batch")
    ap.add_argument("--timeref-mode", choices=("predictor", "floor"), default="predictor",
                    help="time refinement: later stages from the explicit predictor, or from the previous stage "
                         "value with the SER floor")
    ap.add_argument("--timeref-schemes", default="2,3,4")
    ap.add_argument("--timeref-steps", default="", help="comma list of step counts for every scheme (default: "
                                                      "the per-scheme counts)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU domain decomposition is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    extras = set(EXTRAS) if args.extra == "all" else {x for x in args.extra.split(",") if x}
    unknown = extras - set(EXTRAS)
    if unknown:
        ap.error(f"unknown --extra blocks: {sorted(unknown)}")

    import torch
    from paper_1908_03972_amd import api
    torch.cuda.set_device(0)

    if args.only_extra:
        line, detail = None, {}
    else:
        line, detail = headline_line(api, torch, args)
    if "vortex" in extras or "nk" in extras:
        detail["vortex_64x64_P321_esdirk3"], vlevels, vq0 = vortex_block(
            api, torch, ["mixed", "fp64"], 3, 1, args.vortex_vcycles, args.kernel_reps, not args.no_autotune)
        progress("vortex 64x64")
        if "nk" in extras:
            detail["newton_krylov_vs_fas_64x64_P321_stage"] = newton_krylov_block(api, torch, vlevels, vq0,
                                                                                  ["mixed", "fp64"])
            progress("Newton-Krylov against FAS")
        del vlevels, vq0
    if "small" in extras:
        detail["time_to_1e-8_8x8_P210_esdirk2"] = small_vortex_block(api, torch, ["mixed", "fp64"])
        progress("8x8 time to 1e-8")
    if "airfoil" in extras:
        detail["airfoil_128x64_P4_steady"] = airfoil_block(api, torch, ["mixed", "fp64"], args.airfoil_vcycles,
                                                           args.kernel_reps)
        progress("airfoil steady solves")
    if "lines" in extras:
        detail["airfoil_128x64_P421_element_vs_line_jacobi"] = airfoil_lines_block(api, torch, args.airfoil_vcycles,
                                                                                  args.kernel_reps)
        progress("airfoil element against line Jacobi")
    if "viscous" in extras:
        detail["viscous_batch_256x96"] = viscous_batch_block(api, torch, args.viscous_vcycles)
        progress("viscous batch")
    if "timeref" in extras:
        floor = args.timeref_mode == "floor"
        schemes = tuple(int(x) for x in args.timeref_schemes.split(",") if x)
        steps = ({sc: tuple(int(x) for x in args.timeref_steps.split(",")) for sc in schemes}
                 if args.timeref_steps else None)
        detail["time_refinement_vortex50_P5"] = time_refinement_block(
            api, torch, schemes=schemes, steps=steps, later_guess="previous" if floor else "predictor",
            ser_floor=floor)
    if "sphere2" in extras:
        detail["sphere_cubed_16x16x24_P2_steady"] = sphere_block(api, torch, ["mixed", "fp64"], args.sphere_vcycles,
                                                                 args.kernel_reps)
        progress("sphere P{2-1-0}")
    if line is not None and not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
        progress("cpu baseline")
    if args.detail:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
            with open(args.detail, "w") as fh:
                json.dump({"line": line, **detail}, fh, indent=1)
        except OSError as e:
            print(f"bench: could not write {args.detail}: {e}", file=sys.stderr)
    for k, v in detail.items():
        if k != "headline":
            print(f"bench: {k}: {json.dumps(v)}", file=sys.stderr, flush=True)
    if line is not None:
        print(json.dumps(line), flush=True)


def headline_line(api, torch, args):
    """The headline solves and the compact bench line built from them."""
    head = sphere_headline(api, torch, args.steps, args.warmup, args.fp64_solves, args.max_vcycles,
                           args.kernel_reps, autotune=not args.no_autotune)
    mx, f64 = head["mixed"], head.get("fp64")
    achieved = mx["sweep_bytes"] / (mx["sweep_ms"] * 1e-3) / 1e9
    n0 = 5 * (HEAD_PLEV[0] + 1) ** 3
    traffic = measured_traffic(PROFILE_PMC_SPHERE3, KERNEL_SOURCES_3D)
    if mx["elements_per_workgroup"][0] != 4:       # the counters were taken with 4 elements per workgroup
        traffic = None
    t_mx = mx["ms_per_solve"] * 1e-3
    t_64 = f64["ms_per_solve"] * 1e-3 if f64 else None
    line = {
        "metric": METRIC,
        "value": mx["dof_updates_per_s"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 residual/update + f32 block solves",
        "data": "synthetic",
        "config": {"workload": "steady Ma 0.001 flow past the unit sphere, cubed sphere 6x16x16x24 quadratic hexes "
                               "(36864), P{3-2-1-0} I{5-10-20-20}, CFL 30->1e5, solve from free stream to 1e-8 drop",
                   "elements": head["elements"], "dof_fine": head["dof_fine"],
                   "dof_updates_per_vcycle": head["dof_updates_per_vcycle"], "form": "mixed, graph replay"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fr3<3,2> fine-level fused residual + element-Jacobi sweep (FP32 blocks)",
                     "kernel_ms": mx["sweep_ms"], "bytes_per_launch": mx["sweep_bytes"],
                     "bytes_per_dof_update": 4 * n0 + 24},
        "time_to_1e-8_s": {"mixed": t_mx, "fp64": t_64},
        "speedup_time_to_1e-8_mixed_over_fp64": (t_64 / t_mx) if t_64 else None,
        "vcycles_per_solve": {"mixed": mx["vcycles"][0], "fp64": f64["vcycles"][0] if f64 else None},
        "converged": all(s == 0 for s in mx["status"]) and (f64 is None or all(s == 0 for s in f64["status"])),
        "fp64_form": ({"dof_updates_per_s": f64["dof_updates_per_s"], "sweep_ms": f64["sweep_ms"],
                       "sweep_frac": f64["sweep_bytes"] / (f64["sweep_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "solves": f64["solves"]} if f64 else None),
        "mixed_vs_fp64_rel_err_max": max(head["mixed_vs_fp64_rel_err"]) if "mixed_vs_fp64_rel_err" in head else None,
        "fine_rebuild": {"ms_mixed": mx["rebuild_ms"], "ms_fp64": f64["rebuild_ms"] if f64 else None,
                         "tflops_2n3_per_element_mixed": head["elements"] * 2.0 * n0 ** 3 / (mx["rebuild_ms"] * 1e-3) / 1e12},
    }
    return line, {"headline": head}


if __name__ == "__main__":
    main()
