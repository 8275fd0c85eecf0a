"""Batches of independent cases (esdirk_step_batched, esdirk_stage_solve_batched): running cases
together on the batch's streams must give, case by case and bit for bit, what the single-case
entry points give (no case may see another's data)."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle.fr import FRLevel

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402
from paper_1908_03972_amd import _abi as A  # noqa: E402

VS = W.VortexSpec(length=10.0)
FS = W.FreeStreamSpec(ma_inf=0.01)


def vortex_case(mesh, plev, nsm, prec, graph):
    qinf = VS.freestream()
    levels = [api.Level(mesh, P, gamma=VS.gamma, rgas=VS.rgas, eps_mode=0, ma_inf=VS.ma_inf, q_inf=qinf, q_ref=qinf)
              for P in plev]
    olev = FRLevel(mesh, plev[0], OG.Gas(gamma=VS.gamma, rgas=VS.rgas))
    q0 = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1]) - qinf
    make = lambda: api.StageSolver(levels, [api.Factors(lv, prec) for lv in levels], nsm, tol_rel=1e-6,  # noqa
                                   max_vcycles=8, use_graph=graph)
    return levels, to_dev(q0), make


def viscous_channel_case(plev, nsm):
    mesh = W.channel_mesh(9, 5, 6.0, 2.0, jitter=0.1, seed=4)
    qinf = FS.freestream()
    levels = [api.Level(mesh, P, gamma=FS.gamma, rgas=FS.rgas, eps_mode=1, ma_inf=FS.ma_inf, kappa=1.0, q_inf=qinf,
                        q_ref=qinf, mu=2e-3) for P in plev]
    olev = FRLevel(mesh, plev[0], OG.Gas())
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    dq = np.zeros(x.shape + (4,))
    dq[..., 1] = 0.1 * np.sin(0.7 * x) * np.cos(0.5 * y)
    dq[..., 3] = 0.05 * np.cos(0.9 * x + 0.3 * y)
    make = lambda: api.StageSolver(levels, [api.Factors(lv, 64) for lv in levels], nsm, tol_rel=1e-6,  # noqa
                                   max_vcycles=8, use_cfl=True, cfl_init=1e2, cfl_max=1e4)
    return levels, to_dev(dq), make


def build_cases():
    return [vortex_case(W.periodic_quad_mesh(8, 10.0), (2, 1, 0), (5, 10, 20), 64, True),
            vortex_case(W.periodic_rect_mesh(13, 11, 10.0, 10.0, jitter=0.1, seed=3), (3, 1), (3, 6), 32, False),
            viscous_channel_case((3, 2, 1), (3, 6, 10))]


def test_batched_esdirk_step_matches_single_cases():
    cases = build_cases()
    dts = [0.05, 0.05, 0.02]
    stages = api.esdirk_stages(3)
    # single-case runs
    singles, single_stats = [], []
    for (levels, q0, make), dt in zip(cases, dts):
        q = q0.clone()
        work = torch.zeros((stages,) + levels[0].shape, dtype=torch.float64, device="cuda")
        single_stats.append(api.esdirk_step(make(), 3, dt, q, work, raise_on_error=False))
        singles.append(q.cpu().numpy())
    # the same cases as one batch (fresh solver objects, same levels)
    solvers = [make() for (_, _, make) in cases]
    batch = api.Batch(solvers)
    qs = [q0.clone() for (_, q0, _) in cases]
    works = [torch.zeros((stages,) + lv[0].shape, dtype=torch.float64, device="cuda") for (lv, _, _) in cases]
    bstats = batch.esdirk_step(3, dts, qs, works, raise_on_error=False)
    torch.cuda.synchronize()
    for c in range(len(cases)):
        assert np.array_equal(qs[c].cpu().numpy(), singles[c]), c
        assert [s["n_vcycles"] for s in bstats[c]] == [s["n_vcycles"] for s in single_stats[c]]
        assert [s["history"] for s in bstats[c]] == [s["history"] for s in single_stats[c]]
    batch.close()


def test_batched_stage_solve_mixes_steady_and_unsteady():
    cases = build_cases()
    # case 0 unsteady (ESDIRK2 second stage), cases 1 and 2 steady
    levels0, q00, make0 = cases[0]
    g = OG.Gas(gamma=VS.gamma, rgas=VS.rgas)
    olev = FRLevel(W.periodic_quad_mesh(8, 10.0), 2, g)
    qa = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    gam = 1 - 2 ** -0.5
    qc, R1 = to_dev(OG.conservative(qa, g)), to_dev(olev.residual(qa))
    single = []
    for c, (lv, q0, make) in enumerate(cases):
        q = q0.clone()
        if c == 0:
            single.append(make().solve(q, omega=gam, dt=0.05, qc_n=qc, R_prev=[R1], a_row=[gam], raise_on_error=False))
        else:
            single.append(make().solve(q, raise_on_error=False))
        single[-1]["q"] = q.cpu().numpy()
    batch = api.Batch([make() for (_, _, make) in cases])
    qs = [q0.clone() for (_, q0, _) in cases]
    out = batch.solve(qs, omega=[gam, 0.0, 0.0], dt=[0.05, None, None], qc_n=[qc, None, None],
                      R_prev=[[R1], None, None], a_row=[[gam], None, None], raise_on_error=False)
    torch.cuda.synchronize()
    for c in range(len(cases)):
        assert out[c]["history"] == single[c]["history"], c
        assert np.array_equal(qs[c].cpu().numpy(), single[c]["q"]), c
    batch.close()


def test_a_failing_case_does_not_stop_the_others():
    """A case whose input holds a NaN stops with PMG_E_NONFINITE; the other cases of the batch
    finish their step exactly as they would alone."""
    cases = build_cases()
    stages = api.esdirk_stages(2)
    bad_levels, bad_q, bad_make = vortex_case(W.periodic_quad_mesh(6, 10.0), (2, 1), (3, 6), 64, False)
    bad_q = bad_q.clone()
    bad_q[0, 0, 0] = float("nan")
    all_cases = cases + [(bad_levels, bad_q, bad_make)]
    singles = []
    for (levels, q0, make) in cases:
        q = q0.clone()
        work = torch.zeros((stages,) + levels[0].shape, dtype=torch.float64, device="cuda")
        api.esdirk_step(make(), 2, 0.05, q, work, raise_on_error=False)
        singles.append(q.cpu().numpy())
    batch = api.Batch([make() for (_, _, make) in all_cases])
    qs = [q0.clone() for (_, q0, _) in all_cases]
    works = [torch.zeros((stages,) + lv[0].shape, dtype=torch.float64, device="cuda") for (lv, _, _) in all_cases]
    st = batch.esdirk_step(2, [0.05] * 4, qs, works, raise_on_error=False)
    torch.cuda.synchronize()
    assert st[3][0]["status"] == A.PMG_E_NONFINITE and st[3][1]["status"] == A.PMG_E_NONFINITE
    for c in range(3):
        assert np.array_equal(qs[c].cpu().numpy(), singles[c]), c
    batch.close()


def test_batch_rejects_shared_levels():
    levels, _, make = build_cases()[0]
    s1, s2 = make(), make()
    opts = (A.SolveOpts * 2)(s1.opts, s2.opts)
    h = A.pmg_batch()
    assert A.lib().pmg_batch_create(opts, 2, h) == A.PMG_E_ARG


def test_batched_cases_against_the_oracle():
    """Two cases in one batch, each checked against the CPU oracle (not only against its own
    single-case run): the 8x8 vortex at P{2-1-0} with FP64 blocks on an ESDIRK2 second stage, and
    the ragged 13x11 jittered vortex at P{3-1} with FP32 blocks, steady; three V-cycles each,
    within ten times the oracle's own one-ulp floor (FP64) or FP32-rounding floor (FP32)."""
    from oracle import solver as OS
    from gpu_helpers import fp32_solver_class, from_dev, rel_err_per_var
    g = OG.Gas(gamma=VS.gamma, rgas=VS.rgas, eps_mode="local", ma_inf=VS.ma_inf)
    qinf = VS.freestream()
    mesh_a, mesh_b = W.periodic_quad_mesh(8, 10.0), W.periodic_rect_mesh(13, 11, 10.0, 10.0, jitter=0.1, seed=3)
    (la, qa0, _), (lb, qb0, _) = (vortex_case(mesh_a, (2, 1, 0), (5, 10, 20), 64, True),
                                  vortex_case(mesh_b, (3, 1), (3, 6), 32, False))
    gam, dt, nvc = 1 - 2 ** -0.5, 0.05, 3
    olev = FRLevel(mesh_a, 2, g, q_inf=qinf)
    qa = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    src = (OG.conservative(qa, g) + dt * gam * olev.residual(qa)) / (gam * dt)
    qb = from_dev(qb0) + qinf

    def oracle(mesh, plev, nsm, q0, cls=OS.PMGSolver, unsteady=False):
        sol = cls(mesh, g, OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30), q_inf=qinf)
        if unsteady:
            return sol.stage_solve(q0, 1.0 / (gam * dt), src)
        return sol.stage_solve(q0)

    rng = np.random.default_rng(5)
    ra, _ = oracle(mesh_a, (2, 1, 0), (5, 10, 20), qa, unsteady=True)
    ra_p, _ = oracle(mesh_a, (2, 1, 0), (5, 10, 20), qa * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=qa.shape)),
                     unsteady=True)
    rb, _ = oracle(mesh_b, (3, 1), (3, 6), qb)
    rb_p, _ = oracle(mesh_b, (3, 1), (3, 6), qb, cls=fp32_solver_class())
    mk = lambda lv, prec, graph: api.StageSolver(lv, [api.Factors(x, prec) for x in lv],  # noqa
                                                  (5, 10, 20) if len(lv) == 3 else (3, 6), tol_rel=1e-30,
                                                  max_vcycles=nvc, use_graph=graph)
    batch = api.Batch([mk(la, 64, True), mk(lb, 32, False)])
    qs = [qa0.clone(), qb0.clone()]
    out = batch.solve(qs, omega=[gam, 0.0], dt=[dt, None], qc_n=[to_dev(OG.conservative(qa, g)), None],
                      R_prev=[[to_dev(olev.residual(qa))], None], a_row=[[gam], None], raise_on_error=False)
    torch.cuda.synchronize()
    assert [o["n_vcycles"] for o in out] == [nvc, nvc]
    for q, ref, pert in ((qs[0], ra, ra_p), (qs[1], rb, rb_p)):
        err = rel_err_per_var(from_dev(q), ref - qinf)
        floor = rel_err_per_var(pert - qinf, ref - qinf)
        print("batched case err", err, "floor", floor)
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    batch.close()


def test_batched_cases_against_the_oracle():
    """Two FP64 cases of different mesh size and hierarchy solved together as one batch (the 8 x 8
    P{2-1-0} and the ragged 13 x 11 P{3-1} vortex, ESDIRK2 second stage, three V-cycles each):
    every case's state and residual history against the oracle's stage solve, within ten times the
    oracle's own one-ulp floor, as the single-case solves are tested."""
    from gpu_helpers import from_dev, rel_err_per_var
    from oracle import solver as OS
    g = OG.Gas(gamma=VS.gamma, rgas=VS.rgas, eps_mode="local", ma_inf=VS.ma_inf)
    qinf = VS.freestream()
    A2 = OS.esdirk_tableau("esdirk2")
    dt, om = 0.05, A2[1, 1]
    specs = [(W.periodic_quad_mesh(8, 10.0), (2, 1, 0), (5, 10, 20)),
             (W.periodic_rect_mesh(13, 11, 10.0, 10.0, jitter=0.1, seed=3), (3, 1), (3, 6))]
    nvc = 3
    solvers, qs, qcs, R1s, refs = [], [], [], [], []
    for mesh, plev, nsm in specs:
        olev = FRLevel(mesh, plev[0], g, q_inf=qinf)
        q0 = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])

        def run_oracle(x, mesh=mesh, plev=plev, nsm=nsm):
            osol = OS.PMGSolver(mesh, g, OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30),
                                q_inf=qinf)
            src = (OG.conservative(x, g) + dt * A2[1, 0] * osol.levels[0].residual(x)) / (om * dt)
            return osol.stage_solve(x, 1.0 / (om * dt), src, max_vcycles=nvc)

        q_ref, st = run_oracle(q0)
        rng = np.random.default_rng(7)
        q_pert, _ = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
        refs.append((q_ref, st, rel_err_per_var(q_pert - qinf, q_ref - qinf)))
        levels = [api.Level(mesh, P, gamma=VS.gamma, rgas=VS.rgas, eps_mode=0, ma_inf=VS.ma_inf, q_inf=qinf,
                            q_ref=qinf) for P in plev]
        solvers.append(api.StageSolver(levels, [api.Factors(lv, 64) for lv in levels], nsm, max_vcycles=nvc,
                                       tol_rel=1e-30))
        qs.append(to_dev(q0 - qinf))
        qcs.append(to_dev(OG.conservative(q0, g)))
        R1s.append(to_dev(olev.residual(q0)))
    batch = api.Batch(solvers)
    out = batch.solve(qs, omega=[om, om], dt=[dt, dt], qc_n=qcs, R_prev=[[R1s[0]], [R1s[1]]],
                      a_row=[[A2[1, 0]], [A2[1, 0]]], raise_on_error=False)
    torch.cuda.synchronize()
    for c, (q_ref, st, floor) in enumerate(refs):
        assert out[c]["n_vcycles"] == nvc
        err = rel_err_per_var(from_dev(qs[c]), q_ref - qinf)
        h_ref = np.array(st.history)
        h_err = np.abs(np.array(out[c]["history"]) - h_ref) / h_ref
        print("batched case", c, "state err", err, "floor", floor, "history err", h_err)
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (c, err, floor)
        assert np.all(h_err <= max(1e-11, 10.0 * floor.max())), (c, h_err)
    batch.close()
