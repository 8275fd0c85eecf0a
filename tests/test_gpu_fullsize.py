"""GPU (HIP through the C ABI) against the CPU oracle on the full-size workloads, in the launch
configuration the benchmark times: the 64x64 jittered vortex mesh (4096 elements, P{3-2-1}, Sec. 4.1
setting), the 128x64 airfoil O-mesh (8192 elements, P4, Sec. 4.2 setting) and the 256x96 viscous
O-mesh (24576 elements, P4 with BR2, Sec. 4.3 setting).

Residuals and P-transfers are compared at every point. Element blocks and sweeps are compared on
sampled elements (wall, far-field, trailing-edge and seeded random ones): the oracle evaluates each
sampled element's block on a patch made of the element and its face neighbours, which yields the
same block as the whole mesh because the block holds the neighbours' states fixed (Sec. 2.4,
eq. (30)); the sweep update of a sampled element is the oracle's solve with that block and the
whole-mesh stage residual."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr import FRLevel

from gpu_helpers import fp32_inverse, from_dev, rel_err_per_var, rounding_floor, to_dev, tolerance
from patches import patch_block

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

ESDIRK3_GAMMA = 0.4358665215084590   # diagonal coefficient of the three-stage ESDIRK scheme


def scaled_block_error(got, ref, qe, qinf):
    """Block difference as responses to relative perturbations of each unknown (column scale
    max(|q_j|, 1e-3 of the free-stream magnitude of its variable)), relative to the row maximum."""
    scale = np.maximum(np.abs(qe).ravel(), np.tile(np.abs(qinf) * 1e-3, qe.shape[0]))
    rowmax = np.max(np.abs(ref) * scale[None, :], axis=1, keepdims=True)
    return float(np.max(np.abs(got - ref) * scale[None, :] / rowmax))


def sampled_update_check(D, F, F_ulp, dq_gpu, prec, seed=3, fp32_elimination=False):
    """Sweep update of one element against the oracle's solve D dq = F. The bound is ten times
    what the same rounding does to the oracle: the stage residual from a state moved by one ulp
    (F_ulp; at low Mach number the residual amplifies rounding), and a one-ulp perturbation of D
    (FP64 blocks) or the inverse rounded to FP32, or computed in FP32 where the GPU eliminates in
    FP32 (P4), and applied in FP32 (FP32 blocks)."""
    ref = np.linalg.solve(D, F)
    if prec == 64:
        rng = np.random.default_rng(seed)
        alt = np.linalg.solve(D * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=D.shape)), F)
    else:
        inv32 = fp32_inverse(D) if fp32_elimination else np.linalg.inv(D)
        alt = (inv32.astype(np.float32) @ F.astype(np.float32)).astype(np.float64)
    nv = 4
    err = rel_err_per_var(dq_gpu.reshape(-1, nv), ref.reshape(-1, nv))
    floor = np.maximum(rel_err_per_var(alt.reshape(-1, nv), ref.reshape(-1, nv)),
                       rel_err_per_var(np.linalg.solve(D, F_ulp).reshape(-1, nv), ref.reshape(-1, nv)))
    return err, floor


def ulp_moved(q, seed=1):
    rng = np.random.default_rng(seed)
    return q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape))


# ---------------------------------------------------------------------------------------------
# the 64x64 vortex, P{3-2-1}


@pytest.fixture(scope="module")
def vortex():
    mesh, vs = W.vortex_config2()
    gas = OG.Gas(gamma=vs.gamma, rgas=vs.rgas, eps_mode="local", ma_inf=vs.ma_inf)
    return mesh, vs, gas


def vortex_level(mesh, vs, P):
    qinf = vs.freestream()
    return api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf, q_inf=qinf, q_ref=qinf)


@pytest.mark.parametrize("P", [3, 2, 1])
def test_vortex_fullsize_residual(vortex, P):
    mesh, vs, gas = vortex
    olev = FRLevel(mesh, P, gas, q_inf=vs.freestream())
    glev = vortex_level(mesh, vs, P)
    xy = olev.geo.xy
    q = vs.state(xy[..., 0], xy[..., 1])
    c_mass = 1.0 / (ESDIRK3_GAMMA * 0.05)
    src = c_mass * OG.conservative(q, gas) * (1.0 + 1e-3 * np.sin(xy[..., :1]))

    def fun(x):
        return olev.stage_residual(x, c_mass=c_mass, src=src)

    ref = fun(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - vs.freestream()), F, src=to_dev(src), c_mass=c_mass)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    tol = tolerance(rounding_floor(fun, q))
    print("vortex P", P, "err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


def test_vortex_fullsize_transfers(vortex):
    mesh, vs, gas = vortex
    rng = np.random.default_rng(17)
    lv = {P: vortex_level(mesh, vs, P) for P in (3, 2, 1)}
    for Pf, Pc in ((3, 2), (2, 1)):
        xf = rng.standard_normal((mesh.n_elements, (Pf + 1) ** 2, 4))
        xc = lv[Pc].new_state()
        api.pmg_restrict(lv[Pf], lv[Pc], to_dev(xf), xc)
        dc = rng.standard_normal((mesh.n_elements, (Pc + 1) ** 2, 4))
        xo = to_dev(xf)
        api.pmg_prolong(lv[Pc], lv[Pf], to_dev(dc), xo)
        torch.cuda.synchronize()
        assert np.all(rel_err_per_var(from_dev(xc), OS.restrict(xf, Pf, Pc)) < 1e-13)
        assert np.all(rel_err_per_var(from_dev(xo), xf + OS.prolong(dc, Pc, Pf)) < 1e-13)


@pytest.mark.parametrize("prec,dtau", [(32, 10.0), (64, 0.01)])
def test_vortex_fullsize_blocks_and_sweep(vortex, prec, dtau):
    """Fine-level (P3) blocks and one sweep of the ESDIRK3 stage residual, sampled elements."""
    mesh, vs, gas = vortex
    P = 3
    qinf = vs.freestream()
    olev = FRLevel(mesh, P, gas, q_inf=qinf)
    glev = vortex_level(mesh, vs, P)
    xy = olev.geo.xy
    q = vs.state(xy[..., 0], xy[..., 1])
    c_mass = 1.0 / (ESDIRK3_GAMMA * 0.05)
    src = c_mass * OG.conservative(q, gas) * (1.0 + 1e-3 * np.cos(xy[..., :1]))
    F = olev.stage_residual(q, c_mass=c_mass, src=src)
    F_ulp = olev.stage_residual(ulp_moved(q), c_mass=c_mass, src=src)
    fac = api.Factors(glev, prec)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    qd = to_dev(q - qinf)
    api.fr_element_jacobian(glev, qd, dtau, c_mass, fac, D_out=D)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1, src=to_dev(src), c_mass=c_mass)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0)
    sample = np.random.default_rng(2019).choice(mesh.n_elements, 6, replace=False).tolist() + [0, 4095]
    Dg = D.view(glev.ne, glev.n, glev.n)
    for e in sample:
        Dref = patch_block(mesh, gas, P, q, e, dtau, c_mass, qinf)
        berr = scaled_block_error(Dg[e].cpu().numpy(), Dref, q[e], qinf)
        err, floor = sampled_update_check(Dref, F[e].ravel(), F_ulp[e].ravel(), dq[e], prec)
        print("vortex e", e, "block err", berr, "update err", err, "floor", floor)
        assert berr < 1e-12
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (e, err, floor)


def test_vortex_fullsize_stage_vcycles(vortex):
    """Two V-cycles of the first implicit ESDIRK3 stage on the whole 64x64 vortex mesh, P{3-2-1},
    I{5-10-20}, dtau 0.01 -> 10, FP64 blocks, the V-cycles replayed from a HIP graph as the
    benchmark runs them: the state after each V-cycle and the residual history against the
    oracle, within ten times the oracle's own response to a one-ulp change of the start."""
    mesh, vs, gas = vortex
    plev, nsm, nvc = (3, 2, 1), (5, 10, 20), 2
    qinf = vs.freestream()
    A = OS.esdirk_tableau("esdirk3")
    om, dt = A[1, 1], 0.05
    olev = FRLevel(mesh, 3, gas, q_inf=qinf)
    q0 = vs.state(olev.geo.xy[..., 0], olev.geo.xy[..., 1])
    R0 = olev.residual(q0)
    src = (OG.conservative(q0, gas) + dt * A[1, 0] * R0) / (om * dt)

    def run(qs):
        sol = OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30),
                           q_inf=qinf)
        return sol.stage_solve(qs, 1.0 / (om * dt), src)

    q_ref, st = run(q0)
    q_pert, st_pert = run(ulp_moved(q0, 4))
    floor = rel_err_per_var(q_pert - qinf, q_ref - qinf)
    h_ref = np.array(st.history)
    h_floor = np.max(np.abs(np.array(st_pert.history) - h_ref) / h_ref)
    levels = [vortex_level(mesh, vs, P) for P in plev]
    solver = api.StageSolver(levels, [api.Factors(lv, 64) for lv in levels], nsm, max_vcycles=nvc, tol_rel=1e-30,
                             use_graph=True)
    q = to_dev(q0 - qinf)
    out = solver.solve(q, omega=om, dt=dt, qc_n=to_dev(OG.conservative(q0, gas)), R_prev=[to_dev(R0)],
                       a_row=[A[1, 0]], raise_on_error=False)
    torch.cuda.synchronize()
    assert out["n_vcycles"] == nvc
    err = rel_err_per_var(from_dev(q), q_ref - qinf)
    h_err = np.abs(np.array(out["history"]) - h_ref) / h_ref
    print("vortex 64x64 V-cycles err", err, "floor", floor, "history err", h_err, "floor", h_floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-11, 10.0 * h_floor))


# ---------------------------------------------------------------------------------------------
# the 128x64 airfoil O-mesh, P4, steady


@pytest.fixture(scope="module")
def airfoil():
    mesh, fs = W.airfoil_config3()
    gas = OG.Gas(gamma=fs.gamma, rgas=fs.rgas, eps_mode="cutoff", ma_inf=fs.ma_inf, kappa=1.0)
    return mesh, fs, gas


def airfoil_level(mesh, fs, P):
    qinf = fs.freestream()
    return api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0, q_inf=qinf,
                     q_ref=qinf)


def airfoil_state(olev, qinf, gamma):
    """Free stream plus a smooth disturbance of the size a Ma 0.001 flow carries."""
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    q = np.broadcast_to(qinf, x.shape + (4,)).copy()
    s = np.sin(0.7 * x) * np.cos(0.5 * y) / (1.0 + 0.05 * (x * x + y * y))
    q[..., 0] += 0.8 * s
    q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
    q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
    q[..., 3] += 0.8 * s / qinf[0] * qinf[3] * (gamma - 1) / gamma
    return q


def airfoil_sample(n_wrap, n_radial, seed):
    wall = [0, 1, n_wrap // 2, n_wrap - 1]                       # trailing edge, leading edge
    far = [(n_radial - 1) * n_wrap + 5, n_radial * n_wrap - 1]
    rnd = np.random.default_rng(seed).choice(n_wrap * n_radial, 4, replace=False).tolist()
    return wall + far + rnd


def test_airfoil_fullsize_residual(airfoil):
    mesh, fs, gas = airfoil
    qinf = fs.freestream()
    olev = FRLevel(mesh, 4, gas, q_inf=qinf)
    glev = airfoil_level(mesh, fs, 4)
    q = airfoil_state(olev, qinf, fs.gamma)
    ref = olev.residual(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - qinf), F)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    tol = tolerance(rounding_floor(olev.residual, q))
    print("airfoil P4 err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


@pytest.mark.parametrize("prec", [32, 64])
def test_airfoil_fullsize_blocks_and_sweep(airfoil, prec):
    mesh, fs, gas = airfoil
    P = 4
    qinf = fs.freestream()
    olev = FRLevel(mesh, P, gas, q_inf=qinf)
    glev = airfoil_level(mesh, fs, P)
    q = airfoil_state(olev, qinf, fs.gamma)
    dtau = 600.0 * OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=(P,), n_smooth=(1,)), q_inf=qinf).dtau_min(q)
    F = olev.residual(q)
    F_ulp = olev.residual(ulp_moved(q))
    fac = api.Factors(glev, prec)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    qd = to_dev(q - qinf)
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac, D_out=D)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0)
    Dg = D.view(glev.ne, glev.n, glev.n)
    for e in airfoil_sample(128, 64, 4):
        Dref = patch_block(mesh, gas, P, q, e, dtau, 0.0, qinf)
        berr = scaled_block_error(Dg[e].cpu().numpy(), Dref, q[e], qinf)
        err, floor = sampled_update_check(Dref, F[e].ravel(), F_ulp[e].ravel(), dq[e], prec,
                                          fp32_elimination=True)
        print("airfoil e", e, "block err", berr, "update err", err, "floor", floor)
        assert berr < 1e-12
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (e, err, floor)


# ---------------------------------------------------------------------------------------------
# the 256x96 viscous O-mesh, P4, BR2, first case of the batch


@pytest.fixture(scope="module")
def viscous():
    mesh, cases = W.viscous_config4()
    c = next(c for c in cases if c.P == 4)
    gas = OG.Gas(gamma=c.spec.gamma, rgas=c.spec.rgas, eps_mode="cutoff", ma_inf=c.spec.ma_inf, kappa=1.0, mu=c.mu,
                 prandtl=c.prandtl)
    return mesh, c, gas


def viscous_level(mesh, c, P):
    qinf = c.spec.freestream()
    return api.Level(mesh, P, gamma=c.spec.gamma, rgas=c.spec.rgas, eps_mode=1, ma_inf=c.spec.ma_inf, kappa=1.0,
                     q_inf=qinf, q_ref=qinf, mu=c.mu, prandtl=c.prandtl)


def test_viscous_fullsize_residual(viscous):
    mesh, c, gas = viscous
    qinf = c.spec.freestream()
    olev = FRLevel(mesh, 4, gas, q_inf=qinf)
    glev = viscous_level(mesh, c, 4)
    q = W.viscous_start_state(c.spec, olev.geo.xy)
    ref = olev.residual(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - qinf), F)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    # the floor of the viscous residual needs a second whole-mesh evaluation (~4 s)
    tol = tolerance(rounding_floor(olev.residual, q))
    print("viscous P4 err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


def test_viscous_fullsize_blocks_and_sweep(viscous):
    mesh, c, gas = viscous
    P, prec = 4, 32
    qinf = c.spec.freestream()
    olev = FRLevel(mesh, P, gas, q_inf=qinf)
    glev = viscous_level(mesh, c, P)
    q = W.viscous_start_state(c.spec, olev.geo.xy)
    c_mass = 1.0 / (ESDIRK3_GAMMA * 0.05)
    src = c_mass * OG.conservative(q, gas)
    F = olev.stage_residual(q, c_mass=c_mass, src=src)
    F_ulp = olev.stage_residual(ulp_moved(q), c_mass=c_mass, src=src)
    dtau = 10.0 * OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=(P,), n_smooth=(1,)), q_inf=qinf).dtau_min(q)
    fac = api.Factors(glev, prec)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    qd = to_dev(q - qinf)
    api.fr_element_jacobian(glev, qd, dtau, c_mass, fac, D_out=D)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1, src=to_dev(src), c_mass=c_mass)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0)
    Dg = D.view(glev.ne, glev.n, glev.n)
    for e in airfoil_sample(256, 96, 5):
        Dref = patch_block(mesh, gas, P, q, e, dtau, c_mass, qinf)
        berr = scaled_block_error(Dg[e].cpu().numpy(), Dref, q[e], qinf)
        err, floor = sampled_update_check(Dref, F[e].ravel(), F_ulp[e].ravel(), dq[e], prec,
                                          fp32_elimination=True)
        print("viscous e", e, "block err", berr, "update err", err, "floor", floor)
        assert berr < 1e-11
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (e, err, floor)
