"""Lookahead of the single-case stage solve (pmg_solve_opts.lookahead): the V-cycle after the one in
flight is enqueued before the host reads its norm, and discarded (the state restored) when the
stopping test says stop. Whatever the mode, the solve must give bit for bit the state, the norm
history, the V-cycle count and the rebuild count of the plain loop (lookahead 0): on a solve that
converges (the speculative V-cycle then in flight and dropped), one that runs into max_vcycles,
rebuilds every few V-cycles, with and without graph replay, FP64 and FP32 blocks, and whole
ESDIRK steps."""
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

VS = W.VortexSpec(length=10.0)


GAM = 1 - 2 ** -0.5   # ESDIRK2 diagonal: the second stage of a step of 0.05 from the vortex


def vortex_levels(mesh, plev):
    qinf = VS.freestream()
    levels = [api.Level(mesh, P, gamma=VS.gamma, rgas=VS.rgas, eps_mode=0, ma_inf=VS.ma_inf, q_inf=qinf, q_ref=qinf)
              for P in plev]
    g = OG.Gas(gamma=VS.gamma, rgas=VS.rgas)
    olev = FRLevel(mesh, plev[0], g)
    qa = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    stage = (to_dev(OG.conservative(qa, g)), to_dev(olev.residual(qa)))
    return levels, to_dev(qa - qinf), stage


def solve(levels, q0, stage, nsm, prec, lookahead, **kw):
    facs = [api.Factors(lv, prec) for lv in levels]
    solver = api.StageSolver(levels, facs, nsm, lookahead=lookahead, **kw)
    q = q0.clone()
    qc, R1 = stage
    st = solver.solve(q, omega=GAM, dt=0.05, qc_n=qc, R_prev=[R1], a_row=[GAM], raise_on_error=False)
    torch.cuda.synchronize()
    return q.cpu().numpy(), st


def same(a, b):
    qa, sa = a
    qb, sb = b
    assert np.array_equal(qa, qb)
    for k in ("status", "n_vcycles", "n_refresh", "history", "r0", "r_final"):
        assert sa[k] == sb[k], k


CASES = [  # mesh, P levels, smoothing, block precision, graph replay
    (lambda: W.periodic_quad_mesh(8, 10.0), (2, 1, 0), (5, 10, 20), 64, True),
    (lambda: W.periodic_rect_mesh(13, 11, 10.0, 10.0, jitter=0.1, seed=3), (3, 1), (3, 6), 32, True),
    (lambda: W.periodic_quad_mesh(8, 10.0), (2, 1), (4, 8), 64, False),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lookahead_converging_solve_matches_plain_loop(case):
    mk, plev, nsm, prec, graph = CASES[case]
    levels, q0, stage = vortex_levels(mk(), plev)
    kw = dict(dtau_init=0.01, dtau_max=10.0, refresh_every=100, use_graph=graph)
    # the plain loop's history over 12 V-cycles sets a tolerance that it meets after a few of them
    _, probe = solve(levels, q0, stage, nsm, prec, 0, tol_rel=1e-30, max_vcycles=12, **kw)
    h = np.asarray(probe["history"])
    tol = float(h[1:9].min() / h[0]) * (1.0 + 1e-9)
    ref = solve(levels, q0, stage, nsm, prec, 0, tol_rel=tol, max_vcycles=12, **kw)
    assert ref[1]["status"] == 0 and ref[1]["n_vcycles"] >= 1
    for la in (1, 2):
        same(solve(levels, q0, stage, nsm, prec, la, tol_rel=tol, max_vcycles=12, **kw), ref)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lookahead_to_max_vcycles_with_rebuilds_matches_plain_loop(case):
    mk, plev, nsm, prec, graph = CASES[case]
    levels, q0, stage = vortex_levels(mk(), plev)
    kw = dict(dtau_init=0.01, dtau_max=10.0, refresh_every=3, freeze_at_max=False, use_graph=graph, tol_rel=1e-30,
              max_vcycles=10)
    ref = solve(levels, q0, stage, nsm, prec, 0, **kw)
    assert ref[1]["n_vcycles"] == 10 and ref[1]["n_refresh"] >= 4
    for la in (1, 2):
        same(solve(levels, q0, stage, nsm, prec, la, **kw), ref)


def test_lookahead_esdirk_step_matches_plain_loop():
    levels, q0, _ = vortex_levels(W.periodic_quad_mesh(8, 10.0), (2, 1, 0))
    out = {}
    for la in (0, 2):
        facs = [api.Factors(lv, 32) for lv in levels]
        solver = api.StageSolver(levels, facs, (5, 10, 20), dtau_init=0.01, dtau_max=10.0, refresh_every=4,
                                 tol_rel=1e-5, max_vcycles=30, use_graph=True, lookahead=la)
        q = q0.clone()
        work = torch.zeros((api.esdirk_stages(3),) + levels[0].shape, dtype=torch.float64, device="cuda")
        st = api.esdirk_step(solver, 3, 0.05, q, work, raise_on_error=False)
        torch.cuda.synchronize()
        out[la] = (q.cpu().numpy(), st)
    assert np.array_equal(out[0][0], out[2][0])
    for a, b in zip(out[0][1], out[2][1]):
        for k in ("status", "n_vcycles", "n_refresh", "history"):
            assert a[k] == b[k], k
