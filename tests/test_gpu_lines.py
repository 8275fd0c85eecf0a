"""GPU (HIP through the C ABI) against the CPU oracle for element-line Jacobi (``oracle.lines``):
the coupling blocks, line sweeps and V-cycles on a small O-mesh around the profile (radial lines
from the wall to the far field, and lines round the profile across the periodic seam), and the
full-size 128 x 64 O-mesh at P4 on sampled lines and elements."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import lines as OL
from oracle import solver as OS
from oracle.fr import FRLevel

from gpu_helpers import fp32_solver_class, from_dev, rel_err_per_var, to_dev
from patches import patch_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

FS = W.FreeStreamSpec()
QINF = FS.freestream()
GAS = OG.Gas(gamma=FS.gamma, rgas=FS.rgas, eps_mode="cutoff", ma_inf=FS.ma_inf, kappa=1.0)
NW, NR = 16, 8


def small_mesh():
    """16 x 8 cells: 16 radial lines of 8 elements."""
    return W.airfoil_o_mesh(NW, NR, ratio=1.3, r_far=10.0)


def radial_lines(nw, nr):
    return np.arange(nw)[:, None] + nw * np.arange(nr)[None, :]


def wrap_lines(nw, nr):
    """Lines round the profile, one per layer, open at the periodic seam between i = nw-1 and 0."""
    return np.arange(nw)[None, :] + nw * np.arange(nr)[:, None]


def glevel(mesh, P):
    return api.Level(mesh, P, gamma=FS.gamma, rgas=FS.rgas, eps_mode=1, ma_inf=FS.ma_inf, kappa=1.0,
                     q_inf=QINF, q_ref=QINF)


def disturbed(olev, seed=0):
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    q = np.broadcast_to(QINF, x.shape + (4,)).copy()
    s = np.sin(0.7 * x + 0.3 * seed) * np.cos(0.5 * y)
    q[..., 0] += 0.8 * s
    q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
    q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
    q[..., 3] += 0.8 * s / QINF[0] * QINF[3] * (FS.gamma - 1) / FS.gamma
    return q


def scaled_block_error(got, ref, q_cols):
    """Block difference as responses to relative perturbations of each unknown the block acts on
    (column scale max(|q_j|, 1e-3 of the free-stream magnitude)), relative to the row maximum of
    the reference (rows that are zero in the reference must be zero)."""
    scale = np.maximum(np.abs(q_cols).ravel(), np.tile(np.abs(QINF) * 1e-3, q_cols.shape[0]))
    rowmax = np.max(np.abs(ref) * scale[None, :], axis=1, keepdims=True)
    if np.all(rowmax == 0.0):
        return float(np.max(np.abs(got)))
    return float(np.max(np.abs(got - ref) * scale[None, :] / np.maximum(rowmax, 1e-300)))


def thomas(D, Am, Ap, line, b, w_dtype=np.float64):
    """Block Thomas on one line with the inverses W_k applied at w_dtype (products in FP64): what
    FP32 storage of W does to the line solve, to size the parity bound."""
    K = len(line)
    Wi, y = [], []
    for k, e in enumerate(line):
        Dk = D[e] - (Am[e] @ Wi[k - 1] @ Ap[line[k - 1]] if k else 0.0)
        Wi.append(np.linalg.inv(Dk))
    Wa = [w.astype(w_dtype).astype(np.float64) for w in Wi]
    for k, e in enumerate(line):
        y.append(Wa[k] @ (b[k] - (Am[e] @ y[k - 1] if k else 0.0)))
    x = [None] * K
    for k in reversed(range(K)):
        x[k] = y[k] - (Wa[k] @ Ap[line[k]] @ x[k + 1] if k + 1 < K else 0.0)
    return np.array(x)


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_line_blocks_parity(P):
    """D_e, and the blocks towards the previous and next element of each radial line."""
    mesh = small_mesh()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev, 1)
    lines = radial_lines(NW, NR)
    dtau, c_mass = 0.05, 3.0
    D, Am, Ap = OL.line_blocks(olev, q, dtau, c_mass, lines)
    fac = api.LineFactors(glev, lines, 64)
    Dg, Amg, Apg = (from_blk.cpu().numpy() for from_blk in api.line_blocks(fac, to_dev(q - QINF), dtau, c_mass))
    torch.cuda.synchronize()
    assert glev.status() == 0
    prev = np.full(mesh.n_elements, -1)
    nxt = np.full(mesh.n_elements, -1)
    prev[lines[:, 1:]] = lines[:, :-1]
    nxt[lines[:, :-1]] = lines[:, 1:]
    worst = [0.0, 0.0, 0.0]
    for e in range(mesh.n_elements):
        worst[0] = max(worst[0], scaled_block_error(Dg[e], D[e], q[e]))
        if prev[e] >= 0:
            worst[1] = max(worst[1], scaled_block_error(Amg[e], Am[e], q[prev[e]]))
        else:
            assert np.all(Amg[e] == 0.0)
        if nxt[e] >= 0:
            worst[2] = max(worst[2], scaled_block_error(Apg[e], Ap[e], q[nxt[e]]))
        else:
            assert np.all(Apg[e] == 0.0)
    print("P", P, "block errors D, Am, Ap", worst)
    assert max(worst) < 1e-12


@pytest.mark.parametrize("P,prec,kind", [(1, 64, "radial"), (2, 64, "radial"), (3, 64, "radial"),
                                         (4, 64, "radial"), (4, 32, "radial"), (2, 64, "wrap"),
                                         (3, 32, "wrap"), (0, 32, "ragged"), (1, 32, "ragged"),
                                         (1, 64, "ragged"), (2, 32, "ragged")])
def test_line_sweep_parity(P, prec, kind):
    """Three steady line sweeps at pseudo-time step 1e3 dtau_min. The bound is ten times the
    oracle's own response to a one-ulp change of the state (FP64), or to W_k rounded to FP32 in a
    block-Thomas solve with the oracle's blocks (FP32), and at least 1e-11. "ragged": radial lines
    on a 13 x 7 O-mesh, whose 91 elements leave the last workgroup of the substitution kernels
    partly empty at every grouping (64, 8, 4 or 3 elements per workgroup at P0-P2)."""
    nw, nr = (13, 7) if kind == "ragged" else (NW, NR)
    mesh = W.airfoil_o_mesh(nw, nr, ratio=1.3, r_far=10.0) if kind == "ragged" else small_mesh()
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    lines = radial_lines(nw, nr) if kind in ("radial", "ragged") else wrap_lines(nw, nr)
    q = disturbed(olev, 3)
    dtau = 1e3 * OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(1,)), q_inf=QINF).dtau_min(q)
    blocks = OL.line_blocks(olev, q, dtau, 0.0, lines)
    ref = OL.line_sweeps(olev, q, blocks, lines, 3)
    if prec == 64:
        rng = np.random.default_rng(11)
        qp = q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape))
        alt = OL.line_sweeps(olev, qp, OL.line_blocks(olev, qp, dtau, 0.0, lines), lines, 3)
    else:
        alt = q.copy()
        for _ in range(3):
            F = olev.stage_residual(alt).reshape(olev.ne, olev.n)
            dq = np.zeros_like(F)
            for line in lines:
                dq[line] = thomas(*blocks, line, F[line], np.float32)
            alt = alt + dq.reshape(alt.shape)
    floor = rel_err_per_var(alt - QINF, ref - QINF)
    fac = api.LineFactors(glev, lines, prec)
    qd = to_dev(q - QINF)
    api.fr_element_jacobian(glev, qd, dtau, 0.0, fac)
    api.ejacobi_sweep(glev, fac, qd, 3)
    torch.cuda.synchronize()
    assert glev.status() == 0
    err = rel_err_per_var(from_dev(qd), ref - QINF)
    print("line sweep P", P, prec, kind, "err", err, "floor", floor)
    assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (err, floor)


def test_lines_of_one_element_sweep_like_element_jacobi():
    """Lines of length one: the line sweep is the element-Jacobi sweep of eq. (30). Both GPU paths
    (FP64) against the oracle's element-Jacobi sweeps, within ten times the oracle's response to a
    one-ulp change of the state (the temperature update amplifies rounding at Ma 0.001)."""
    mesh = small_mesh()
    P = 3
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    q = disturbed(olev, 5)
    dtau = 0.02

    def oracle_sweeps(q0):
        sol = OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(2,)), q_inf=QINF)
        sol.c_mass, sol.src, sol.dtau = 0.0, None, dtau
        sol.build_D(0, q0)
        return sol.smooth(0, q0, None, 2)

    ref = oracle_sweeps(q)
    rng = np.random.default_rng(2)
    floor = rel_err_per_var(oracle_sweeps(q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape))) - QINF,
                            ref - QINF)
    q_line = to_dev(q - QINF)
    q_elem = q_line.clone()
    lf = api.LineFactors(glev, np.arange(mesh.n_elements)[:, None], 64)
    ef = api.Factors(glev, 64)
    api.fr_element_jacobian(glev, q_line, dtau, 0.0, lf)
    api.fr_element_jacobian(glev, q_elem, dtau, 0.0, ef)
    api.ejacobi_sweep(glev, lf, q_line, 2)
    api.ejacobi_sweep(glev, ef, q_elem, 2)
    torch.cuda.synchronize()
    err_line = rel_err_per_var(from_dev(q_line), ref - QINF)
    err_elem = rel_err_per_var(from_dev(q_elem), ref - QINF)
    print("length-one lines", err_line, "element Jacobi", err_elem, "floor", floor)
    bound = np.maximum(1e-11, 10.0 * floor)
    assert np.all(err_line <= bound) and np.all(err_elem <= bound), (err_line, err_elem, floor)


def fp32_line_solver_class():
    """The oracle's solver with FP32 smoother inverses: element levels as in ``fp32_solver_class``,
    line levels by block Thomas with W_k rounded to FP32 (the elimination in FP64), the rounding
    the GPU's FP32 line factors introduce."""
    base = fp32_solver_class()

    class PMGSolverLinesFP32(base):
        def smooth(self, l, q, S, nsweep):
            lines = self.level_lines(l)
            if lines is None:
                return super().smooth(l, q, S, nsweep)
            lev = self.levels[l]
            for _ in range(nsweep):
                F = self.F(l, q, S).reshape(lev.ne, lev.n)
                dq = np.zeros_like(F)
                for line in lines:
                    dq[line] = thomas(*self.D[l], line, F[line], np.float32)
                q = q + self.opts.alpha_r * dq.reshape(q.shape)
            return q

    return PMGSolverLinesFP32


@pytest.mark.parametrize("plev,nsm,line_levels,prec", [((3, 2, 1), (3, 4, 8), (0,), 64),
                                                       ((3, 2, 1), (3, 4, 8), (0, 1, 2), 64),
                                                       ((4, 2, 1), (3, 4, 8), (0,), 32)])
def test_line_vcycle_parity(plev, nsm, line_levels, prec):
    """Steady V-cycles with the CFL form (1e2 -> 1e5), line Jacobi on the listed levels and element
    Jacobi elsewhere: state and residual history after 3 V-cycles against the oracle."""
    mesh = small_mesh()
    nvc = 3
    lines = radial_lines(NW, NR)
    per_level = tuple(lines if l in line_levels else None for l in range(len(plev)))

    def run_oracle(q0, cls=OS.PMGSolver):
        opts = OS.PMGOptions(p_levels=plev, n_smooth=nsm, max_vcycles=nvc, tol=1e-30, use_cfl=True,
                             cfl_init=1e2, cfl_max=1e5, lines=per_level)
        return cls(mesh, GAS, opts, q_inf=QINF).stage_solve(q0)

    q0 = disturbed(FRLevel(mesh, plev[0], GAS, q_inf=QINF), 4)
    q_ref, st = run_oracle(q0)
    if prec == 64:
        rng = np.random.default_rng(7)
        q_pert, st_pert = run_oracle(q0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q0.shape)))
    else:
        q_pert, st_pert = run_oracle(q0, fp32_line_solver_class())
    floor = rel_err_per_var(q_pert - QINF, q_ref - QINF)
    h_floor = np.max(np.abs(np.array(st_pert.history) - np.array(st.history)) / np.array(st.history))
    glevels = [glevel(mesh, P) for P in plev]
    facs = [api.LineFactors(lv, lines, prec) if l in line_levels else api.Factors(lv, prec)
            for l, lv in enumerate(glevels)]
    solver = api.StageSolver(glevels, facs, nsm, max_vcycles=nvc, tol_rel=1e-30, use_cfl=True, cfl_init=1e2,
                             cfl_max=1e5)
    q = to_dev(q0 - QINF)
    out = solver.solve(q, raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == -6 and out["n_vcycles"] == nvc
    err = rel_err_per_var(from_dev(q), q_ref - QINF)
    h_err = np.abs(np.array(out["history"]) - np.array(st.history)) / np.array(st.history)
    # ten times the oracle's response to a one-ulp change of the start (FP64) or to FP32 inverses
    bound = np.maximum(1e-11, 10.0 * floor)
    print(plev, line_levels, prec, "state err", err, "floor", floor, "history err", h_err, "floor", h_floor)
    assert np.all(err <= bound), (err, floor)
    assert np.all(h_err <= max(float(bound.max()), 10.0 * h_floor))


def test_line_factors_reject_bad_lines():
    mesh = small_mesh()
    glev = glevel(mesh, 1)
    with pytest.raises(api.A.PmgError):
        api.LineFactors(glev, np.arange(mesh.n_elements).reshape(2, -1))      # not neighbours at the row ends
    with pytest.raises(api.A.PmgError):
        api.LineFactors(glev, np.zeros((mesh.n_elements, 1)))                # repeated elements
    with pytest.raises(api.A.PmgError):
        api.LineFactors(glev, radial_lines(NW, NR)[:, :4])                   # not every element
    with pytest.raises(api.A.PmgError):
        api.LineFactors(glevel(mesh, 5), radial_lines(NW, NR))               # P > 4


# ---------------------------------------------------------------------------------------------
# the 128 x 64 O-mesh at P4, in the launch configuration the benchmark times


@pytest.mark.parametrize("prec", [64, 32])
def test_airfoil_fullsize_line_blocks_and_sweep(prec):
    """128 radial lines of 64 elements. Sampled elements' coupling blocks against the oracle on a
    patch (the element and its face neighbours give the same blocks as the whole mesh); one line
    sweep on sampled lines against the dense solve of the line's block-tridiagonal system built
    from the GPU's blocks, the bound being ten times what W_k rounded to FP32 (FP32) or a one-ulp
    change of the blocks (FP64) does to the oracle's solve."""
    mesh, fs = W.airfoil_config3()
    P, nw, nr = 4, 128, 64
    olev = FRLevel(mesh, P, GAS, q_inf=QINF)
    glev = glevel(mesh, P)
    x, y = olev.geo.xy[..., 0], olev.geo.xy[..., 1]
    q = np.broadcast_to(QINF, x.shape + (4,)).copy()
    s = np.sin(0.7 * x) * np.cos(0.5 * y) / (1.0 + 0.05 * (x * x + y * y))
    q[..., 0] += 0.8 * s
    q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
    q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
    q[..., 3] += 0.8 * s / QINF[0] * QINF[3] * (FS.gamma - 1) / FS.gamma
    dtau = 600.0 * OS.PMGSolver(mesh, GAS, OS.PMGOptions(p_levels=(P,), n_smooth=(1,)), q_inf=QINF).dtau_min(q)
    lines = radial_lines(nw, nr)
    fac = api.LineFactors(glev, lines, prec)
    qd = to_dev(q - QINF)
    D, Am, Ap = api.line_blocks(fac, qd, dtau, 0.0)
    F = glev.new_state()
    api.fr_residual(glev, qd, F)
    q0 = qd.clone()
    api.ejacobi_sweep(glev, fac, qd, 1)
    torch.cuda.synchronize()
    assert glev.status() == 0
    dq = from_dev(qd - q0).reshape(glev.ne, glev.n)
    r = from_dev(F).reshape(glev.ne, glev.n)
    # sampled coupling blocks against the oracle on patches
    for e in (lines[0, 0], lines[0, 1], lines[64, 31], lines[127, 62], lines[5, 63]):
        pm, elems = patch_mesh(mesh, int(e))
        plev = FRLevel(pm, P, GAS, q_inf=QINF)
        for k_side, blk in ((0, Am), (1, Ap)):
            pos = int(np.where(lines[e % nw] == e)[0][0])
            other = pos - 1 if k_side == 0 else pos + 1
            got = blk[int(e)].cpu().numpy()
            if not 0 <= other < nr:
                assert np.all(got == 0.0)
                continue
            nb = int(lines[e % nw][other])
            f = OL.face_towards(mesh, int(e), nb)
            ref = OL.neighbour_blocks(plev, q[elems], f)[0]
            berr = scaled_block_error(got, ref, q[nb])
            print("e", e, "side", k_side, "block err", berr)
            assert berr < 1e-12
    # sampled line sweeps against the dense solve with the GPU's blocks
    for li in (0, 64, 101):
        line = lines[li]
        Dl, Aml, Apl = (t[torch.as_tensor(line, device=t.device)].cpu().numpy() for t in (D, Am, Ap))
        loc = np.arange(nr)
        ref = OL.line_solve(Dl, Aml, Apl, loc, r[line])
        if prec == 64:
            rng = np.random.default_rng(li)
            pert = [b * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=b.shape)) for b in (Dl, Aml, Apl)]
            alt = OL.line_solve(*pert, loc, r[line])
        else:
            alt = thomas(Dl, Aml, Apl, loc, r[line], np.float32)
        err = rel_err_per_var(dq[line].reshape(-1, 4), ref.reshape(-1, 4))
        floor = rel_err_per_var(alt.reshape(-1, 4), ref.reshape(-1, 4))
        print("line", li, prec, "err", err, "floor", floor)
        assert np.all(err <= np.maximum(1e-11, 10.0 * floor)), (li, err, floor)
