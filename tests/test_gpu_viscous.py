"""GPU (HIP through the C ABI) against the CPU oracle with the BR2 viscous terms (Sec. 2.1 fluxes,
Sec. 2.3 eqs. (22)-(23)): residuals, element blocks, sweeps and V-cycles on a channel between
no-slip adiabatic walls and on a viscous airfoil O-mesh."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr import FRLevel
from oracle.jacobian import element_blocks

from gpu_helpers import fp32_solver_class, from_dev, rel_err_per_var, rounding_floor, to_dev, tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

MA = 0.01
QINF = np.array([1.0 / MA ** 2 / 1.4, 1.0, 0.05, 1.0 / MA ** 2 / 1.4])
MU = 2e-3
GAS = OG.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=MA, kappa=1.0, mu=MU, br2_penalty=4.0)


def mesh_of(name):
    if name == "channel":
        return W.channel_mesh(9, 5, 6.0, 2.0, jitter=0.1, seed=4)
    return W.airfoil_o_mesh(16, 6, ratio=1.3, r_far=6.0, wall=W.BC_NOSLIP_WALL)


def glevel(mesh, P):
    return api.Level(mesh, P, gamma=1.4, rgas=1.0, eps_mode=1, ma_inf=MA, kappa=1.0, q_inf=QINF, q_ref=QINF,
                     mu=MU, prandtl=0.72, br2_penalty=4.0)


def disturbed(olev, seed=0):
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    q = np.broadcast_to(QINF, x.shape + (4,)).copy()
    q[..., 0] += 0.3 * np.sin(0.7 * x + 0.3 * seed) * np.cos(0.9 * y)
    q[..., 1] += 0.3 * np.cos(0.9 * x - 0.8 * y + seed)
    q[..., 2] += 0.2 * np.sin(1.1 * y + 0.2 * x)
    q[..., 3] += 0.2 * np.cos(0.5 * x + 0.7 * y)
    return q


@pytest.mark.parametrize("name,P", [("channel", 1), ("channel", 2), ("channel", 3), ("channel", 4),
                                    ("airfoil", 2), ("airfoil", 4), ("channel", 0)])
def test_viscous_residual_parity(name, P):
    mesh = mesh_of(name)
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev)
    ref = olev.residual(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - QINF), F)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    tol = tolerance(rounding_floor(olev.residual, q))
    print(name, P, "err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


def test_viscous_dtau_min():
    mesh = mesh_of("channel")
    glev = glevel(mesh, 3)
    sol = OS.PMGSolver(mesh, OG.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=MA, mu=50.0),
                       OS.PMGOptions(p_levels=(3,), n_smooth=(1,)), q_inf=QINF)
    q = disturbed(sol.levels[0], 1)
    hi = api.Level(mesh, 3, gamma=1.4, rgas=1.0, eps_mode=1, ma_inf=MA, q_inf=QINF, q_ref=QINF, mu=50.0)
    assert abs(api.dtau_min(hi, to_dev(q - QINF)) - sol.dtau_min(q)) <= 1e-13 * sol.dtau_min(q)
    del glev


def scaled_block_error(got, ref, q):
    scale = np.maximum(np.abs(q), np.abs(QINF) * 1e-3)
    sc = scale.reshape(q.shape[0], 1, -1)
    rowmax = np.max(np.abs(ref) * sc, axis=2, keepdims=True)
    return float(np.max(np.abs(got - ref) * sc / rowmax))


@pytest.mark.parametrize("name,P", [("channel", 1), ("channel", 2), ("channel", 3), ("airfoil", 4)])
def test_viscous_element_blocks_parity(name, P):
    mesh = mesh_of(name)
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev, 2)
    dtau, c_mass = 0.05, 46.0
    ref = element_blocks(olev, q, dtau, c_mass)
    fac = api.Factors(glev, 64)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    api.fr_element_jacobian(glev, to_dev(q - QINF), dtau, c_mass, fac, D_out=D)
    torch.cuda.synchronize()
    assert glev.status() == 0
    err = scaled_block_error(D.cpu().numpy().reshape(glev.ne, glev.n, glev.n), ref, q)
    print(name, P, "scaled block err", err)
    assert err < 1e-12


@pytest.mark.parametrize("name,P,prec", [("channel", 3, 64), ("airfoil", 4, 64), ("channel", 3, 32)])
def test_viscous_sweep_parity(name, P, prec):
    mesh = mesh_of(name)
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    c_mass = 1.0 / (0.4358665 * 0.05)           # 1/(omega dt) of ESDIRK3 with dt = 0.05
    q = disturbed(olev, 3)
    src = c_mass * OG.conservative(q, GAS)       # a stage source that leaves F(q) = R(q)

    def oracle_sweeps(q0, cls=OS.PMGSolver):
        sol = cls(mesh, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(3,)), q_inf=QINF)
        sol.c_mass, sol.src, sol.dtau = c_mass, src, 1e2 * sol.dtau_min(q0)
        sol.build_D(0, q0)
        return sol.smooth(0, q0, None, 3), sol.dtau

    ref, dtau = oracle_sweeps(q)
    if prec == 64:
        rng = np.random.default_rng(11)
        ref_pert, _ = oracle_sweeps(q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape)))
    else:
        ref_pert, _ = oracle_sweeps(q, fp32_solver_class())
    floor = rel_err_per_var(ref_pert - QINF, ref - QINF)
    fac = api.Factors(glev, prec)
    qd = to_dev(q - QINF)
    api.fr_element_jacobian(glev, qd, dtau, c_mass, fac)
    api.ejacobi_sweep(glev, fac, qd, 3, src=to_dev(src), c_mass=c_mass)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(qd), ref - QINF)
    print(name, P, prec, "sweep err", err, "floor", floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)


@pytest.mark.parametrize("name,plev,nsm", [("airfoil", (3, 2, 1), (3, 6, 10)), ("channel", (4, 2, 1), (3, 6, 10))])
def test_viscous_stage_solve_parity(name, plev, nsm):
    """Three V-cycles of an ESDIRK3 second-stage solve with no-slip walls (on the small O-mesh,
    P{4-2-1} diverges in the oracle as well, so P4 runs on the channel)."""
    mesh = mesh_of(name)
    nvc = 3
    A = OS.esdirk_tableau("esdirk3")
    dt, om = 0.05, A[1, 1]

    def run(q0):
        opts = OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30, use_cfl=True,
                             cfl_init=1e2, cfl_max=1e5)
        sol = OS.PMGSolver(mesh, GAS, opts, q_inf=QINF)
        lev = sol.levels[0]
        src = (OG.conservative(q0, GAS) + dt * A[1, 0] * lev.residual(q0)) / (om * dt)
        return sol.stage_solve(q0, 1.0 / (om * dt), src)

    olev = FRLevel(mesh, plev[0], GAS, q_inf=QINF)
    q0 = disturbed(olev, 4)
    q_ref, st = run(q0)
    rng = np.random.default_rng(7)
    q_pert, _ = run(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    floor = rel_err_per_var(q_pert - QINF, q_ref - QINF)
    glevels = [glevel(mesh, P) for P in plev]
    facs = [api.Factors(lv, 64) for lv in glevels]
    solver = api.StageSolver(glevels, facs, nsm, max_vcycles=nvc, tol_rel=1e-30, use_cfl=True, cfl_init=1e2,
                             cfl_max=1e5)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, omega=om, dt=dt, qc_n=to_dev(OG.conservative(q0, GAS)),
                       R_prev=[to_dev(olev.residual(q0))], a_row=[A[1, 0]], raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    err = rel_err_per_var(from_dev(q), q_ref - QINF)
    h_ref = np.array(st.history)
    h_err = np.abs(np.array(out["history"]) - h_ref) / h_ref
    print(plev, "state err", err, "floor", floor, "history err", h_err)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-11, 10.0 * floor.max()))


@pytest.mark.parametrize("plev,nsm", [((4, 3, 2, 1), (3, 6, 10, 10)), ((2, 1, 0), (3, 6, 10))])
def test_viscous_fp32_vcycles_as_benchmarked(plev, nsm):
    """The viscous batch's form: FP32 element blocks, the hierarchies used for P4 and P2 cases
    ({4-3-2-1}, {2-1-0}) on a no-slip O-mesh, CFL 1 -> 1e2; three V-cycles of an ESDIRK3
    second-stage solve against the oracle, within ten times the deviation that FP32 block
    inverses and products cause in the oracle itself."""
    mesh = mesh_of("airfoil")
    nvc = 3
    A = OS.esdirk_tableau("esdirk3")
    dt, om = 0.05, A[1, 1]
    kw = dict(use_cfl=True, cfl_init=1.0, cfl_max=1e2)

    def run(q0, cls=OS.PMGSolver):
        sol = cls(mesh, GAS, OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30, **kw), q_inf=QINF)
        lev = sol.levels[0]
        src = (OG.conservative(q0, GAS) + dt * A[1, 0] * lev.residual(q0)) / (om * dt)
        return sol.stage_solve(q0, 1.0 / (om * dt), src)

    olev = FRLevel(mesh, plev[0], GAS, q_inf=QINF)
    q0 = disturbed(olev, 5)
    q_ref, st = run(q0)
    q_pert, st_pert = run(q0, fp32_solver_class(fp32_elimination=lambda p: p == 4))
    floor = rel_err_per_var(q_pert - QINF, q_ref - QINF)
    h_ref = np.array(st.history)
    h_floor = np.max(np.abs(np.array(st_pert.history) - h_ref) / h_ref)
    glevels = [glevel(mesh, P) for P in plev]
    facs = [api.Factors(lv, 32) for lv in glevels]
    solver = api.StageSolver(glevels, facs, nsm, max_vcycles=nvc, tol_rel=1e-30, use_graph=True, **kw)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, omega=om, dt=dt, qc_n=to_dev(OG.conservative(q0, GAS)),
                       R_prev=[to_dev(olev.residual(q0))], a_row=[A[1, 0]], raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    err = rel_err_per_var(from_dev(q), q_ref - QINF)
    h_err = np.abs(np.array(out["history"]) - h_ref) / h_ref
    print(plev, "FP32 state err", err, "floor", floor, "history err", h_err, "floor", h_floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-11, 10.0 * h_floor))
