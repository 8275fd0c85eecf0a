"""GPU (HIP through the C ABI) against the CPU oracle on hexahedral levels (Sec. 2.3 in three
dimensions, the sphere setting of Sec. 4.2): a small cubed sphere with rotated elements (every face
orientation code occurs), slip wall on the sphere and far field outside, Ma 0.01 and Ma 0.001 with
the cut-off reference velocity, P = 0..3 (P = 3 blocks, n = 320, on a smaller sphere of 48 elements);
then the full 6 x 16 x 16 x 24 mesh on sampled elements at P = 2 and P = 3."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr3 import FRLevel3
from oracle.geometry3d import element_dx3
from oracle.jacobian import element_blocks

from gpu_helpers import fp32_inverse, fp32_solver_class, from_dev, rel_err_per_var, rounding_floor, to_dev, tolerance
from patches import patch_block
from test_oracle_3d import rotated, small_sphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

FS = W.FreeStream3Spec(ma_inf=0.01)
QINF = FS.freestream()
GAS = OG.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=FS.ma_inf, kappa=1.0)


def glevel(mesh, P, fs=FS):
    qinf = fs.freestream()
    return api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0, q_inf=qinf,
                     q_ref=qinf)


def disturbed(olev, qinf, seed=0):
    return disturbed_at(olev.geo.xyz, qinf, seed)


def disturbed_at(x, qinf, seed=0):
    q = np.broadcast_to(qinf, x.shape[:2] + (5,)).copy()
    s = np.sin(0.7 * x[..., 0] + 0.3 * seed) * np.cos(0.5 * x[..., 1]) * np.cos(0.4 * x[..., 2])
    q[..., 0] += 0.8 * s
    q[..., 1] += 0.2 * np.cos(0.9 * x[..., 0] - 0.4 * x[..., 2])
    q[..., 2] += 0.15 * np.sin(0.6 * x[..., 1] + 0.2 * x[..., 0])
    q[..., 3] += 0.1 * np.cos(0.5 * x[..., 2] + 0.3 * x[..., 1])
    q[..., 4] += 0.8 * s / qinf[0] * qinf[4] * 0.4 / 1.4
    return q


def scaled_block_error(got, ref, q):
    scale = np.maximum(np.abs(q), np.abs(QINF) * 1e-3)
    sc = scale.reshape(q.shape[0], 1, -1)
    rowmax = np.max(np.abs(ref) * sc, axis=2, keepdims=True)
    return float(np.max(np.abs(got - ref) * sc / rowmax))


@pytest.fixture(scope="module")
def sphere():
    return small_sphere(inner=W.BC_SLIP_WALL)


@pytest.fixture(scope="module")
def tiny_sphere():
    """6 x 2 x 2 x 2 hexes with rotated elements: the P = 3 cases, whose oracle blocks (320 x 320)
    are slow to assemble."""
    m = W.cubed_sphere_mesh(2, 2, ratio=1.3, r_far=4.0, inner=W.BC_SLIP_WALL)
    return rotated(m, [0, 5, 11, 20, 26, 33, 38, 41, 44, 47, 13, 30], W.BC_SLIP_WALL)


def pick(request, P, big=3):
    return request.getfixturevalue("tiny_sphere" if P >= big else "sphere")


def test_points_and_element_length(sphere):
    for P in (0, 1, 2):
        olev = FRLevel3(sphere, P, GAS, q_inf=QINF)
        glev = glevel(sphere, P)
        pts = glev.points()
        assert np.max(np.abs(np.moveaxis(pts, 0, -1).transpose(1, 0, 2) - olev.geo.xyz)) < 1e-13 * 4.0
    ref = element_dx3(sphere)
    assert np.max(np.abs(glev.dx() - ref) / ref) < 1e-12


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_residual_parity_3d(sphere, P):
    olev = FRLevel3(sphere, P, GAS, q_inf=QINF)
    glev = glevel(sphere, P)
    q = disturbed(olev, QINF)
    ref = olev.residual(q)
    F = glev.new_state()
    api.fr_residual(glev, to_dev(q - QINF), F)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(F), ref)
    tol = tolerance(rounding_floor(olev.residual, q))
    print("3-D P", P, "err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_freestream_on_gpu_3d(P):
    mesh = small_sphere(inner=W.BC_FAR_FIELD)
    glev = glevel(mesh, P)
    F = glev.new_state()
    api.fr_residual(glev, glev.new_state(), F)        # the free stream itself (zero offset)
    torch.cuda.synchronize()
    Fh = from_dev(F)
    scale = QINF[0] * 10.0
    assert np.max(np.abs(Fh[..., :4])) / scale < 1e-12
    assert np.max(np.abs(Fh[..., 4])) / scale < 1e-12 / FS.ma_inf ** 2


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_element_blocks_parity_3d(request, P):
    sphere = pick(request, P)
    olev = FRLevel3(sphere, P, GAS, q_inf=QINF)
    glev = glevel(sphere, P)
    q = disturbed(olev, QINF, 2)
    dtau, c_mass = 0.05, 3.0
    ref = element_blocks(olev, q, dtau, c_mass)
    fac = api.Factors(glev, 64)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    api.fr_element_jacobian(glev, to_dev(q - QINF), dtau, c_mass, fac, D_out=D)
    torch.cuda.synchronize()
    assert glev.status() == 0
    err = scaled_block_error(D.cpu().numpy().reshape(glev.ne, glev.n, glev.n), ref, q)
    print("3-D P", P, "scaled block err", err)
    assert err < 1e-12


def test_transfers_3d_gpu(sphere):
    rng = np.random.default_rng(9)
    lv = {P: glevel(sphere, P) for P in (3, 2, 1, 0)}
    for Pf, Pc in ((3, 2), (2, 1), (1, 0), (2, 0), (3, 0)):
        xf = rng.standard_normal((sphere.n_elements, (Pf + 1) ** 3, 5))
        xc = lv[Pc].new_state()
        api.pmg_restrict(lv[Pf], lv[Pc], to_dev(xf), xc)
        dc = rng.standard_normal((sphere.n_elements, (Pc + 1) ** 3, 5))
        xo = to_dev(xf)
        api.pmg_prolong(lv[Pc], lv[Pf], to_dev(dc), xo)
        torch.cuda.synchronize()
        ref_c = OS.restrict(xf, Pf, Pc, dim=3)
        ref_f = xf + OS.prolong(dc, Pc, Pf, dim=3)
        assert np.max(np.abs(from_dev(xc) - ref_c)) < 1e-13 * np.max(np.abs(ref_c))
        assert np.max(np.abs(from_dev(xo) - ref_f)) < 1e-13 * np.max(np.abs(ref_f))


@pytest.mark.parametrize("P,prec", [(2, 64), (1, 64), (2, 32), (3, 64), (3, 32)])
def test_sweep_parity_3d(request, P, prec):
    """Three steady element-Jacobi sweeps (eq. (30)) at 1e3 dtau_min."""
    sphere = pick(request, P)
    def oracle_sweeps(q0, cls=OS.PMGSolver):
        sol = cls(sphere, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(3,)), q_inf=QINF)
        sol.c_mass, sol.src, sol.dtau = 0.0, None, 1e3 * sol.dtau_min(q0)
        sol.build_D(0, q0)
        return sol.smooth(0, q0, None, 3), sol.dtau

    olev = FRLevel3(sphere, P, GAS, q_inf=QINF)
    q = disturbed(olev, QINF, 3)
    ref, dtau = oracle_sweeps(q)
    if prec == 64:
        rng = np.random.default_rng(11)
        ref_pert, _ = oracle_sweeps(q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape)))
    else:                                   # FP32 inverses of P >= 2 are eliminated in FP32
        ref_pert, _ = oracle_sweeps(q, fp32_solver_class(fp32_elimination=P >= 2))
    floor = rel_err_per_var(ref_pert - QINF, ref - QINF)
    glev = glevel(sphere, P)
    fac = api.Factors(glev, prec)
    qd = to_dev(q - QINF)
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac)
    api.ejacobi_sweep(glev, fac, qd, 3)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(qd), ref - QINF)
    print("3-D sweep P", P, prec, "err", err, "floor", floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)


@pytest.mark.parametrize("plev,prec", [((2, 1, 0), 64), ((2, 1, 0), 32), ((3, 2, 1, 0), 64), ((3, 2, 1, 0), 32)])
def test_steady_solve_parity_3d(request, plev, prec):
    """Four steady CFL V-cycles of P{2-1-0} and P{3-2-1-0} (CFL 10 -> 1e3; from this start CFL
    1e2 -> 1e5 makes the oracle itself diverge) against the oracle."""
    sphere = pick(request, plev[0])
    nsm, nvc = (3, 6, 10, 10)[:len(plev)], 4

    def run_oracle(q0, cls=OS.PMGSolver):
        opts = OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30, use_cfl=True,
                             cfl_init=10.0, cfl_max=1e3)
        return cls(sphere, GAS, opts, q_inf=QINF).stage_solve(q0)

    q0 = disturbed(FRLevel3(sphere, plev[0], GAS, q_inf=QINF), QINF, 4)
    q_ref, st = run_oracle(q0)
    if prec == 64:
        rng = np.random.default_rng(7)
        q_pert, st_pert = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    else:
        q_pert, st_pert = run_oracle(q0, fp32_solver_class(fp32_elimination=lambda p: p >= 2))
    floor = rel_err_per_var(q_pert - QINF, q_ref - QINF)
    h_floor = np.max(np.abs(np.array(st_pert.history) - np.array(st.history)) / np.array(st.history))
    levels = [glevel(sphere, P) for P in plev]
    facs = [api.Factors(lv, prec) for lv in levels]
    solver = api.StageSolver(levels, facs, nsm, max_vcycles=nvc, tol_rel=1e-30, use_cfl=True, cfl_init=10.0,
                             cfl_max=1e3)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    err = rel_err_per_var(from_dev(q), q_ref - QINF)
    h_err = np.abs(np.array(out["history"]) - np.array(st.history)) / np.array(st.history)
    print("3-D solve", prec, "state err", err, "floor", floor, "history err", h_err, "floor", h_floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)
    assert np.all(h_err <= max(1e-11, 10.0 * floor.max(), 10.0 * h_floor))


# ---- the full-size sphere (6 x 16 x 16 x 24, 36 864 elements), P2, Ma 0.001 ---------------------

def test_sphere_fullsize_residual_blocks_and_sweep():
    mesh, fs = W.sphere_config5()
    qinf = fs.freestream()
    gas = OG.Gas(gamma=fs.gamma, rgas=fs.rgas, eps_mode="cutoff", ma_inf=fs.ma_inf, kappa=1.0)
    P = 2
    olev = FRLevel3(mesh, P, gas, q_inf=qinf)
    glev = glevel(mesh, P, fs)
    q = disturbed(olev, qinf, 5)
    F = olev.residual(q)
    Fg = glev.new_state()
    qd = to_dev(q - qinf)
    api.fr_residual(glev, qd, Fg)
    torch.cuda.synchronize()
    err = rel_err_per_var(from_dev(Fg), F)
    tol = tolerance(rounding_floor(olev.residual, q))
    print("sphere P2 residual err", err, "tol", tol)
    assert np.all(err <= tol), (err, tol)
    dtau = 100.0 * OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=(P,), n_smooth=(1,)), q_inf=qinf).dtau_min(q)
    fac = api.Factors(glev, 32)
    D = torch.zeros(glev.ne * glev.n * glev.n, dtype=torch.float64, device="cuda")
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac, D_out=D)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0)
    Dg = D.view(glev.ne, glev.n, glev.n)
    cells = 6 * 16 * 16
    sample = [0, 255, cells - 1, cells * 23, cells * 24 - 1] + \
        np.random.default_rng(36864).choice(mesh.n_elements, 4, replace=False).tolist()
    for e in sample:
        Dref = patch_block(mesh, gas, P, q, e, dtau, 0.0, qinf)
        berr = scaled_block_error(Dg[e].cpu().numpy()[None], Dref[None], q[e:e + 1])
        ref = np.linalg.solve(Dref, F[e].ravel())
        alt = (fp32_inverse(Dref).astype(np.float32) @ F[e].ravel().astype(np.float32)).astype(np.float64)
        e_err = rel_err_per_var(dq[e], ref.reshape(-1, 5))
        floor = rel_err_per_var(alt.reshape(-1, 5), ref.reshape(-1, 5))
        print("sphere e", e, "block err", berr, "update err", e_err, "floor", floor)
        assert berr < 1e-12
        assert np.all(e_err <= np.maximum(1e-11, 10.0 * floor)), (e, e_err, floor)


def test_sphere_fullsize_p3_residual_and_sweep():
    """P = 3 on the full sphere (n = 320; 15 GB of FP32 inverse blocks): the residual and one
    sweep's update on sampled elements, among them elements that the elimination kernel's
    workgroups take in their later passes over the mesh, against the oracle on each element's
    patch (the element and its face neighbours)."""
    from oracle.fr3 import FRLevel3 as OL3
    from patches import patch_mesh
    mesh, fs = W.sphere_config5()
    qinf = fs.freestream()
    gas = OG.Gas(gamma=fs.gamma, rgas=fs.rgas, eps_mode="cutoff", ma_inf=fs.ma_inf, kappa=1.0)
    P = 3
    glev = glevel(mesh, P, fs)
    x = np.moveaxis(glev.points(), 0, -1).transpose(1, 0, 2)          # [Ne][Np][3]
    q = disturbed_at(x, qinf, 6)
    qd = to_dev(q - qinf)
    Fg = glev.new_state()
    api.fr_residual(glev, qd, Fg)
    torch.cuda.synchronize()
    Fh = from_dev(Fg)
    speed = np.sqrt(fs.gamma * fs.rgas * q[..., 4]) + np.linalg.norm(q[..., 1:4], axis=-1)
    dtau = 100.0 * float(np.min(glev.dx()[:, None] / (P + 1) / speed))
    fac = api.Factors(glev, 32)
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0)
    del fac
    sample = [0, 511, 512, 1023, 1024, 6143, 20000, mesh.n_elements - 1] + \
        np.random.default_rng(36865).choice(mesh.n_elements, 2, replace=False).tolist()
    rng = np.random.default_rng(2)
    for e in sample:
        pm, elems = patch_mesh(mesh, e)
        plev = OL3(pm, P, gas, q_inf=qinf)
        qp = q[elems]
        Fe = plev.residual(qp)[0]
        Fe_pert = plev.residual(qp * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=qp.shape)))[0]
        r_err = rel_err_per_var(Fh[e], Fe)
        r_tol = tolerance(rel_err_per_var(Fe_pert, Fe))
        Dref = patch_block(mesh, gas, P, q, e, dtau, 0.0, qinf)
        ref = np.linalg.solve(Dref, Fe.ravel())
        alt = (fp32_inverse(Dref).astype(np.float32) @ Fe.ravel().astype(np.float32)).astype(np.float64)
        u_err = rel_err_per_var(dq[e], ref.reshape(-1, 5))
        floor = rel_err_per_var(alt.reshape(-1, 5), ref.reshape(-1, 5))
        print("sphere P3 e", e, "residual err", r_err, "tol", r_tol, "update err", u_err, "floor", floor)
        assert np.all(r_err <= r_tol), (e, r_err, r_tol)
        assert np.all(u_err <= np.maximum(1e-11, 10.0 * floor)), (e, u_err, floor)
