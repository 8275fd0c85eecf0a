"""FP64 parity at Ma = 0.3, point by point. At the low Mach numbers of the paper's cases the FP64
residual carries cancellation noise far above 1e-11 (the oracle's own one-ulp floor is 1e-10-1e-8
relative at Ma 0.005), so those parity tests can only bound the GPU by ten times that floor, and a
per-variable 2-norm over the whole field would let an error confined to one element pass diluted.
The kernels' arithmetic does not depend on the Mach number; at Ma 0.3 the floor is 1e-14-4e-13, and
here every point of every element is held to max(1e-11, 10 x floor) relative to the variable's
largest value: the residual (eqs. (20)-(21), (26); 2-D P = 0..6 on the ragged 13 x 11 mesh, whose
143 elements leave every grouping a partial last workgroup, 3-D P = 0..3 on the rotated small
spheres), three FP64 element-Jacobi sweeps (eq. (30)) and three V-cycles of an ESDIRK2 stage solve
(Sec. 3) with the residual history."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr import FRLevel
from oracle.fr3 import FRLevel3

from gpu_helpers import from_dev, to_dev
from test_oracle_3d import rotated, small_sphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

VS = W.VortexSpec(length=10.0, ma_inf=0.3)
QINF = VS.freestream()
GAS = OG.Gas(gamma=VS.gamma, rgas=VS.rgas, eps_mode="local", ma_inf=VS.ma_inf)
FS3 = W.FreeStream3Spec(ma_inf=0.3)
QINF3 = FS3.freestream()
GAS3 = OG.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=FS3.ma_inf, kappa=1.0)
GATE = 1e-11


def ragged():
    return W.periodic_rect_mesh(13, 11, 10.0, 10.0, jitter=0.1, seed=3)


def pointwise(a, ref):
    """Per variable: the largest pointwise difference over the variable's largest |value|."""
    nv = a.shape[-1]
    num = np.abs(a - ref).reshape(-1, nv).max(axis=0)
    return num / np.maximum(np.abs(ref).reshape(-1, nv).max(axis=0), 1e-300)


def one_ulp(q, seed):
    rng = np.random.default_rng(seed)
    return q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape))


def check(name, got, ref, floor):
    tol = np.maximum(GATE, 10.0 * floor)
    err = pointwise(got, ref)
    print(name, "pointwise err", err, "floor", floor)
    assert np.all(err <= tol), (name, err, tol)


def level2(mesh, P):
    return api.Level(mesh, P, gamma=VS.gamma, rgas=VS.rgas, eps_mode=0, ma_inf=VS.ma_inf, q_inf=QINF, q_ref=QINF)


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4, 5, 6])
def test_residual_pointwise_2d(P):
    mesh = ragged()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    q = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    rng = np.random.default_rng(P)
    c_mass = 1.0 / (0.2928932 * 0.05)
    src = OG.conservative(q, GAS) * c_mass * (1 + 1e-3 * rng.standard_normal(q.shape))
    S = 1e-2 * rng.standard_normal(q.shape) * np.abs(src).max(axis=(0, 1))

    def oracle_F(x):
        return olev.stage_residual(x, c_mass, src, S)

    ref = oracle_F(q)
    floor = pointwise(oracle_F(one_ulp(q, 1)), ref)
    glev = level2(mesh, P)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - QINF), F, src=to_dev(src), S=to_dev(S), c_mass=c_mass)
    torch.cuda.synchronize()
    check(f"2-D residual P{P}", from_dev(F), ref, floor)


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_residual_pointwise_3d(P):
    if P == 3:   # 6 x 2 x 2 x 2 hexahedra with rotated elements (the P3 oracle is slow)
        m = W.cubed_sphere_mesh(2, 2, ratio=1.3, r_far=4.0, inner=W.BC_SLIP_WALL)
        mesh = rotated(m, [0, 5, 11, 20, 26, 33, 38, 41, 44, 47, 13, 30], W.BC_SLIP_WALL)
    else:
        mesh = small_sphere(inner=W.BC_SLIP_WALL)
    olev = FRLevel3(mesh, P, GAS3, q_inf=QINF3)
    x = olev.geo.xyz
    q = np.broadcast_to(QINF3, x.shape[:2] + (5,)).copy()
    s = np.sin(0.7 * x[..., 0]) * np.cos(0.5 * x[..., 1]) * np.cos(0.4 * x[..., 2])
    q[..., 0] += 0.2 * s * QINF3[0]
    q[..., 1] += 0.2 * np.cos(0.9 * x[..., 0] - 0.4 * x[..., 2])
    q[..., 2] += 0.15 * np.sin(0.6 * x[..., 1] + 0.2 * x[..., 0])
    q[..., 3] += 0.1 * np.cos(0.5 * x[..., 2] + 0.3 * x[..., 1])
    q[..., 4] += 0.1 * s * QINF3[4]
    ref = olev.residual(q)
    floor = pointwise(olev.residual(one_ulp(q, 2)), ref)
    glev = api.Level(mesh, P, gamma=FS3.gamma, rgas=FS3.rgas, eps_mode=1, ma_inf=FS3.ma_inf, kappa=1.0,
                     q_inf=QINF3, q_ref=QINF3)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - QINF3), F)
    torch.cuda.synchronize()
    check(f"3-D residual P{P}", from_dev(F), ref, floor)


@pytest.mark.parametrize("P", [1, 3, 4])
def test_sweeps_pointwise_fp64(P):
    """Three sweeps with FP64 inverse blocks at dtau 0.05 on the ESDIRK2 stage equation."""
    mesh = ragged()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    q = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    dtau, c_mass = 0.05, 1.0 / (0.2928932 * 0.05)
    src = OG.conservative(q, GAS) * c_mass + olev.residual(q) * (0.2928932 * 0.05 * c_mass)

    def oracle_sweeps(q0):
        sol = OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(3,)), q_inf=QINF)
        sol.c_mass, sol.src, sol.dtau = c_mass, src, dtau
        sol.build_D(0, q0)
        return sol.smooth(0, q0, None, 3)

    ref = oracle_sweeps(q) - QINF
    floor = pointwise(oracle_sweeps(one_ulp(q, 11)) - QINF, ref)
    glev = level2(mesh, P)
    fac = api.Factors(glev, 64)
    qd = to_dev(q - QINF)
    api.fr_element_jacobian(glev, qd, dtau, c_mass, fac)
    api.ejacobi_sweep(glev, fac, qd, 3, src=to_dev(src), c_mass=c_mass)
    torch.cuda.synchronize()
    check(f"2-D FP64 sweeps P{P}", from_dev(qd), ref, floor)


def test_stage_solve_pointwise_fp64():
    """Three V-cycles of P{3-1} I{3-6} on the ESDIRK2 second stage, FP64 blocks: the state point by
    point and every residual norm of the history."""
    mesh = ragged()
    plev, nsm, nvc = (3, 1), (3, 6), 3
    A = OS.esdirk_tableau("esdirk2")
    dt, om = 0.05, A[1, 1]

    def run_oracle(q0):
        osol = OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30),
                            q_inf=QINF)
        lev = osol.levels[0]
        src = (OG.conservative(q0, GAS) + dt * A[1, 0] * lev.residual(q0)) / (om * dt)
        return osol.stage_solve(q0, 1.0 / (om * dt), src, max_vcycles=nvc)

    olev = FRLevel(mesh, plev[0], GAS, q_inf=QINF)
    q0 = VS.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    q_ref, st = run_oracle(q0)
    q_pert, st_pert = run_oracle(one_ulp(q0, 7))
    floor = pointwise(q_pert - QINF, q_ref - QINF)
    h_ref = np.array(st.history)
    h_floor = np.max(np.abs(np.array(st_pert.history) - h_ref) / h_ref)
    levels = [level2(mesh, P) for P in plev]
    solver = api.StageSolver(levels, [api.Factors(lv, 64) for lv in levels], nsm, max_vcycles=nvc, tol_rel=1e-30)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, omega=om, dt=dt, qc_n=to_dev(OG.conservative(q0, GAS)), R_prev=[to_dev(olev.residual(q0))],
                       a_row=[A[1, 0]], raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    check("2-D FP64 stage solve P{3-1}", from_dev(q), q_ref - QINF, floor)
    h_err = np.abs(np.array(out["history"]) - h_ref) / h_ref
    print("history err", h_err, "floor", h_floor)
    assert np.all(h_err <= max(GATE, 10.0 * h_floor)), (h_err, h_floor)
