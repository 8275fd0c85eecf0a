"""GPU (HIP through the C ABI) against the CPU oracle on the curved-wall configuration of Sec. 4.2:
9-node O-mesh around the 12% profile, slip wall and far field, Ma 0.001 with the cut-off
reference velocity (kappa = 1), steady residual (F = R), CFL pseudo time of eqs. (32)-(33)."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr import FRLevel
from oracle.geometry import element_dx
from oracle.jacobian import element_blocks

from gpu_helpers import fp32_solver_class, from_dev, rel_err_per_var, rounding_floor, to_dev, tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

FS = W.FreeStreamSpec()
QINF = FS.freestream()
GAS = OG.Gas(gamma=FS.gamma, rgas=FS.rgas, eps_mode="cutoff", ma_inf=FS.ma_inf, kappa=1.0)


def small_mesh():
    """16 x 8 cells (128 elements: two residual tiles and a ragged tail at every P)."""
    return W.airfoil_o_mesh(16, 8, ratio=1.3, r_far=10.0)


def glevel(mesh, P):
    return api.Level(mesh, P, gamma=FS.gamma, rgas=FS.rgas, eps_mode=1, ma_inf=FS.ma_inf, kappa=1.0,
                     q_inf=QINF, q_ref=QINF)


def disturbed(olev, seed=0):
    """Free stream plus a smooth disturbance of the size a Ma 0.001 flow carries (dp ~ rho |V|^2)."""
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    q = np.broadcast_to(QINF, x.shape + (4,)).copy()
    s = np.sin(0.7 * x + 0.3 * seed) * np.cos(0.5 * y)
    q[..., 0] += 0.8 * s
    q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
    q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
    q[..., 3] += 0.8 * s / QINF[0] * QINF[3] * (FS.gamma - 1) / FS.gamma
    return q


def test_element_length_and_dtau_min():
    mesh = small_mesh()
    glev = glevel(mesh, 4)
    ref = element_dx(mesh)
    assert np.max(np.abs(glev.dx() - ref) / ref) < 1e-13
    sol = OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=(4,), n_smooth=(1,)), q_inf=QINF)
    q = disturbed(sol.levels[0], 1)
    got = api.dtau_min(glev, to_dev(q - QINF))
    assert abs(got - sol.dtau_min(q)) <= 1e-13 * sol.dtau_min(q)


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_airfoil_residual_parity(P):
    mesh = small_mesh()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev)
    ref = olev.residual(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - QINF), F)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    tol = tolerance(rounding_floor(olev.residual, q))
    print("airfoil P", P, "err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


def scaled_block_error(got, ref, q):
    """Blocks compared as responses to relative perturbations of each unknown (column scale
    max(|q_j|, 1e-3 of the free-stream magnitude of its variable))."""
    scale = np.maximum(np.abs(q), np.abs(QINF[:4]) * 1e-3)
    sc = scale.reshape(q.shape[0], 1, -1)
    rowmax = np.max(np.abs(ref) * sc, axis=2, keepdims=True)
    return float(np.max(np.abs(got - ref) * sc / rowmax))


@pytest.mark.parametrize("P", [1, 3, 4])
def test_airfoil_element_blocks_parity(P):
    mesh = small_mesh()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev, 2)
    dtau = 0.05
    ref = element_blocks(olev, q, dtau, 0.0)
    fac = api.Factors(glev, 64)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    api.fr_element_jacobian(glev, to_dev(q - QINF), dtau, 0.0, fac, D_out=D)
    torch.cuda.synchronize()
    assert glev.status() == 0
    err = scaled_block_error(D.cpu().numpy().reshape(glev.ne, glev.n, glev.n), ref, q)
    print("airfoil P", P, "scaled block err", err)
    assert err < 1e-12


@pytest.mark.parametrize("P,prec", [(4, 64), (2, 64), (4, 32)])
def test_airfoil_sweep_parity(P, prec):
    """Three steady element-Jacobi sweeps (eq. (30)) at pseudo-time step 1e3 dtau_min."""
    mesh = small_mesh()
    gas = GAS
    glev = glevel(mesh, P)

    def oracle_sweeps(q0, cls=OS.PMGSolver):
        sol = cls(mesh, gas, OS.PMGOptions(p_levels=(P,), n_smooth=(3,)), q_inf=QINF)
        sol.c_mass, sol.src, sol.dtau = 0.0, None, 1e3 * sol.dtau_min(q0)
        sol.build_D(0, q0)
        return sol.smooth(0, q0, None, 3), sol.dtau

    olev = FRLevel(mesh, P, gas, q_inf=QINF)
    q = disturbed(olev, 3)
    ref, dtau = oracle_sweeps(q)
    if prec == 64:
        rng = np.random.default_rng(11)
        ref_pert, _ = oracle_sweeps(q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape)))
    else:
        ref_pert, _ = oracle_sweeps(q, fp32_solver_class(fp32_elimination=lambda p: p == 4))
    floor = rel_err_per_var(ref_pert - QINF, ref - QINF)
    fac = api.Factors(glev, prec)
    qd = to_dev(q - QINF)
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac)
    api.ejacobi_sweep(glev, fac, qd, 3)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(qd), ref - QINF)
    print("airfoil sweep P", P, prec, "err", err, "floor", floor)
    # FP64: ten times the oracle's own one-ulp response; FP32: ten times the deviation that FP32
    # inverse blocks and FP32 products cause in the oracle
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)


@pytest.mark.parametrize("plev,nsm,prec", [((4, 2, 1), (5, 10, 20), 64), ((4, 3, 2, 1, 0), (5, 10, 20, 20, 20), 64),
                                           ((4, 2, 1), (5, 10, 20), 32)])
def test_airfoil_steady_solve_parity(plev, nsm, prec):
    """Steady V-cycles with the CFL form (1e2 -> 1e5): state and residual history after 4 V-cycles
    against the oracle. The start is a disturbed free stream: at the exact free stream every point
    sits on the kink of the cut-off max(kappa Ma_inf, Ma) (kappa = 1), where rounding picks the
    one-sided derivative of the smoother's Jacobian differently in any two implementations."""
    mesh = small_mesh()
    nvc = 4

    def run_oracle(q0, cls=OS.PMGSolver):
        opts = OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30, use_cfl=True,
                             cfl_init=1e2, cfl_max=1e5)
        return cls(mesh, GAS, opts, q_inf=QINF).stage_solve(q0)

    q0 = disturbed(FRLevel(mesh, plev[0], GAS, q_inf=QINF), 4)
    q_ref, st = run_oracle(q0)
    if prec == 64:
        rng = np.random.default_rng(7)
        q_pert, st_pert = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    else:
        q_pert, st_pert = run_oracle(q0, fp32_solver_class(fp32_elimination=lambda p: p == 4))
    floor = rel_err_per_var(q_pert - QINF, q_ref - QINF)
    h_floor = np.max(np.abs(np.array(st_pert.history) - np.array(st.history)) / np.array(st.history))

    glevels = [glevel(mesh, P) for P in plev]
    facs = [api.Factors(lv, prec) for lv in glevels]
    solver = api.StageSolver(glevels, facs, nsm, max_vcycles=nvc, tol_rel=1e-30, use_cfl=True, cfl_init=1e2,
                             cfl_max=1e5)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    assert abs(out["dtau_min"] * 1e2 - st.dtau_scale[0]) <= 1e-13 * st.dtau_scale[0]
    err = rel_err_per_var(from_dev(q), q_ref - QINF)
    h_ref = np.array(st.history)
    h_err = np.abs(np.array(out["history"]) - h_ref) / h_ref
    print(plev, prec, "state err", err, "floor", floor, "history err", h_err, "floor", h_floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-11, 10.0 * floor.max(), 10.0 * h_floor))
