"""GPU (HIP through the C ABI) against the CPU oracle: the Newton-Krylov stage solve with the
V-cycle as preconditioner (flexible GMRES on the pseudo-transient Newton system of eqs. (27)-(28),
Sec. 5's proposed next step). Three Newton steps of six Krylov directions each on the second
ESDIRK2 stage of the 8x8 vortex, P{2-1-0}, with FP64 and with FP32 blocks in the preconditioner;
then the same stage solved to 1e-8 by both solvers."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS

from gpu_helpers import fp32_solver_class, from_dev, gas_for, rel_err_per_var, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

MESH, VS = W.vortex_config1()
PLEV, NSM = (2, 1, 0), (2, 4, 6)
TAB = OS.esdirk_tableau("esdirk2")
DT, OM = 0.05, TAB[1, 1]


DTAU = dict(dtau_init=10.0, dtau_max=1e4)   # Newton-like steps: the regime the V-cycle preconditions well


def _stage(gas):
    osol = OS.PMGSolver(MESH, gas, OS.PMGOptions(p_levels=PLEV, n_smooth=NSM, tol=1e-30, **DTAU),
                        q_inf=VS.freestream())
    lev = osol.levels[0]
    q0 = VS.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    src = (OG.conservative(q0, gas) + DT * TAB[1, 0] * lev.residual(q0)) / (OM * DT)
    return lev, q0, src


def _gpu(prec, q0, gas, **kw):
    qinf = VS.freestream()
    levels = [api.Level(MESH, P, gamma=VS.gamma, rgas=VS.rgas, eps_mode=0, ma_inf=VS.ma_inf, q_inf=qinf,
                        q_ref=qinf) for P in PLEV]
    facs = [api.Factors(lv, prec) for lv in levels]
    solver = api.StageSolver(levels, facs, NSM, tol_rel=kw.pop("tol", 1e-30), max_vcycles=50, **DTAU)
    lev0 = levels[0]
    q = to_dev(q0 - qinf)
    qc = to_dev(OG.conservative(q0, gas))
    from oracle.fr import FRLevel
    R1 = to_dev(FRLevel(MESH, PLEV[0], gas, q_inf=qinf).residual(q0))
    out = api.nk_stage_solve(solver, q, omega=OM, dt=DT, qc_n=qc, R_prev=[R1], a_row=[TAB[1, 0]],
                             raise_on_error=False, **kw)
    torch.cuda.synchronize()
    assert lev0.status() == 0
    return q, out


@pytest.mark.parametrize("prec", [64, 32])
def test_newton_krylov_parity(prec):
    gas = gas_for(VS)
    lev, q0, src = _stage(gas)
    kw = dict(krylov_dim=6, eta=0.0, max_newton=3)

    def run_oracle(q, cls=OS.PMGSolver):
        sol = cls(MESH, gas, OS.PMGOptions(p_levels=PLEV, n_smooth=NSM, tol=1e-30, **DTAU), q_inf=VS.freestream())
        return sol.nk_stage_solve(q, 1.0 / (OM * DT), src, **kw)

    q_ref, st = run_oracle(q0)
    if prec == 64:
        rng = np.random.default_rng(5)
        q_pert, st_p = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    else:
        q_pert, st_p = run_oracle(q0, fp32_solver_class())
    qinf = VS.freestream()
    floor = rel_err_per_var(q_pert - qinf, q_ref - qinf)
    h_floor = np.max(np.abs(np.array(st_p.history) - np.array(st.history)) / np.array(st.history))
    q, out = _gpu(prec, q0, gas, **kw)
    assert out["status"] == -6 and out["n_newton"] == 3 and out["n_krylov"] == 18 == st.krylov
    err = rel_err_per_var(from_dev(q), q_ref - qinf)
    h_err = np.abs(np.array(out["history"]) - np.array(st.history)) / np.array(st.history)
    print("NK", prec, "state err", err, "floor", floor, "history", out["history"], "err", h_err, "floor", h_floor)
    assert np.all(err <= np.maximum(1e-10, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-10, 10.0 * floor.max(), 10.0 * h_floor)), (h_err, h_floor)


@pytest.mark.parametrize("prec", [64, 32])
def test_newton_krylov_solves_the_stage(prec):
    """To 1e-8 with the adaptive GMRES stop (eta 0.05): the oracle's own stage residual of the GPU
    result is below 1e-8 of r_0 (with FP32 blocks only the preconditioner is FP32)."""
    gas = gas_for(VS)
    lev, q0, src = _stage(gas)
    q_nk, out = _gpu(prec, q0, gas, krylov_dim=10, eta=0.05, max_newton=20, tol=1e-8)
    assert out["status"] == 0, out
    qh = from_dev(q_nk) + VS.freestream()
    c_mass = 1.0 / (OM * DT)
    r0 = np.linalg.norm(lev.stage_residual(q0, c_mass, src))
    r = np.linalg.norm(lev.stage_residual(qh, c_mass, src))
    print("NK", prec, "to 1e-8:", out["n_newton"], "Newton steps,", out["n_krylov"], "directions, oracle r/r0", r / r0,
          "history", [h / out["history"][0] for h in out["history"]])
    assert r / r0 < 1.5e-8


def test_newton_krylov_parity_3d():
    """Hexahedra (five variables): two steady Newton steps of six directions on the rotated
    3 x 3 x 2 cubed sphere, P{2-1-0}, Ma 0.01, slip wall, against the oracle."""
    from oracle.fr3 import FRLevel3
    from test_gpu_3d import GAS as GAS3, QINF as QINF3, FS as FS3, disturbed, glevel
    from test_oracle_3d import small_sphere
    mesh = small_sphere(inner=W.BC_SLIP_WALL)
    plev, nsm = (2, 1, 0), (2, 4, 6)
    dt3 = dict(dtau_init=1.0, dtau_max=1e3)
    q0 = disturbed(FRLevel3(mesh, plev[0], GAS3, q_inf=QINF3), QINF3, 8)
    kw = dict(krylov_dim=6, eta=0.0, max_newton=2, fd_rel=1e-4, pc_rel=1e-4)

    def run_oracle(q):
        sol = OS.PMGSolver(mesh, GAS3, OS.PMGOptions(p_levels=plev, n_smooth=nsm, tol=1e-30, **dt3), q_inf=QINF3)
        return sol.nk_stage_solve(q, 0.0, None, **kw)

    q_ref, st = run_oracle(q0)
    rng = np.random.default_rng(6)
    q_pert, st_p = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    floor = rel_err_per_var(q_pert - QINF3, q_ref - QINF3)
    levels = [glevel(mesh, P, FS3) for P in plev]
    facs = [api.Factors(lv, 64) for lv in levels]
    solver = api.StageSolver(levels, facs, nsm, tol_rel=1e-30, max_vcycles=50, **dt3)
    q = to_dev(q0 - QINF3)
    out = api.nk_stage_solve(solver, q, raise_on_error=False, **kw)
    torch.cuda.synchronize()
    assert levels[0].status() == 0
    assert out["n_newton"] == 2 and out["n_krylov"] == 12 == st.krylov
    err = rel_err_per_var(from_dev(q), q_ref - QINF3)
    h_err = np.abs(np.array(out["history"]) - np.array(st.history)) / np.array(st.history)
    print("NK 3-D state err", err, "floor", floor, "history", out["history"], "err", h_err)
    assert np.all(err <= np.maximum(1e-10, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-10, 10.0 * floor.max()))
