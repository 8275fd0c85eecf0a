"""Pins of the oracle's smoother, transfers, FAS V-cycle, pseudo-time control and ESDIRK driver."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle import solver as S
from oracle.fr import FRLevel
from oracle.jacobian import pseudo_time_blocks

GAS = G.Gas(eps_mode="local")


def _vortex(n=3, P=2, length=10.0, jitter=0.1):
    mesh = W.periodic_quad_mesh(n, length, jitter=jitter, seed=5)
    return mesh, W.VortexSpec(length=length)


@pytest.mark.parametrize("Pf,Pc", [(2, 1), (3, 2), (3, 1), (4, 2), (1, 0)])
def test_transfers_exact_on_tensor_polynomials(Pf, Pc):
    mesh, _ = _vortex(2)
    lf, lc = FRLevel(mesh, Pf, GAS), FRLevel(mesh, Pc, GAS)
    xf = np.stack([lf.ops.x[np.arange(lf.npts) % lf.n1], lf.ops.x[np.arange(lf.npts) // lf.n1]], -1)
    xc = np.stack([lc.ops.x[np.arange(lc.npts) % lc.n1], lc.ops.x[np.arange(lc.npts) // lc.n1]], -1)
    for a in range(Pc + 1):
        for b in range(Pc + 1):
            uf = np.broadcast_to((xf[:, 0] ** a * xf[:, 1] ** b)[None, :, None], (lf.ne, lf.npts, 4))
            uc = np.broadcast_to((xc[:, 0] ** a * xc[:, 1] ** b)[None, :, None], (lc.ne, lc.npts, 4))
            assert np.max(np.abs(S.restrict(uf, Pf, Pc) - uc)) < 1e-13
            assert np.max(np.abs(S.prolong(uc, Pc, Pf) - uf)) < 1e-13
    rng = np.random.default_rng(0)
    uc = rng.standard_normal((lc.ne, lc.npts, 4))
    assert np.max(np.abs(S.restrict(S.prolong(uc, Pc, Pf), Pf, Pc) - uc)) < 1e-13


def test_one_sweep_matches_dense_solve_of_fd_blocks():
    """One element-Jacobi sweep (eq. (30)) against numpy.linalg.solve with the diagonal
    blocks of a central-difference global Jacobian plus Gamma/dtau."""
    mesh, vs = _vortex(3, 1)
    opts = S.PMGOptions(p_levels=(1,), n_smooth=(1,), dtau_init=0.5)
    sol = S.PMGSolver(mesh, GAS, opts)
    lev = sol.levels[0]
    q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    c_mass = 1.0 / (0.29 * 0.05)
    sol.c_mass, sol.src, sol.dtau = c_mass, None, 0.5
    sol.build_D(0, q)
    q1 = sol.smooth(0, q, None, 1)
    F = lev.stage_residual(q, c_mass)
    Dfd = pseudo_time_blocks(lev, q, 0.5)
    for e in range(lev.ne):
        for c in range(lev.n):
            p, v = divmod(c, 4)
            h = 1e-4 * abs(q[e, p, v])
            qp, qm = q.copy(), q.copy()
            qp[e, p, v] += h
            qm[e, p, v] -= h
            Dfd[e, :, c] -= (lev.stage_residual(qp, c_mass)[e] - lev.stage_residual(qm, c_mass)[e]).ravel() / (2 * h)
    dq = np.linalg.solve(Dfd, F.reshape(lev.ne, lev.n, 1)).reshape(q.shape)
    err = np.linalg.norm((q1 - q) - dq, axis=(0, 1)) / np.linalg.norm(dq, axis=(0, 1))
    assert np.all(err < 1e-5), err


def test_fas_fixed_point():
    """If q solves F_0(q) = S_0 exactly, a V-cycle leaves it unchanged (eqs. (38)-(45))."""
    mesh, vs = _vortex(3)
    opts = S.PMGOptions(p_levels=(2, 1, 0), n_smooth=(2, 2, 3), dtau_init=0.3)
    sol = S.PMGSolver(mesh, GAS, opts)
    lev = sol.levels[0]
    q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    sol.c_mass, sol.src, sol.dtau = 20.0, None, 0.3
    S0 = lev.stage_residual(q, 20.0)          # manufactured forcing: F_0(q) - S_0 = 0
    sol.refresh_now = True
    sol.build_D(0, q)
    q1 = sol.vcycle(0, q, S0)
    dist = q - vs.freestream()
    assert np.all(np.linalg.norm(q1 - q, axis=(0, 1)) <= 1e-12 * np.linalg.norm(dist, axis=(0, 1)))


def test_vcycle_reduces_stage_residual():
    mesh, vs = W.vortex_config1()
    opts = S.PMGOptions(p_levels=(2, 1, 0), n_smooth=(5, 10, 20), max_vcycles=8)
    sol = S.PMGSolver(mesh, GAS, opts)
    lev = sol.levels[0]
    q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    A = S.esdirk_tableau("esdirk2")
    dt = 0.05
    src = (G.conservative(q, GAS) + dt * A[1, 0] * lev.residual(q)) / (A[1, 1] * dt)
    _, st = sol.stage_solve(q, 1.0 / (A[1, 1] * dt), src, max_vcycles=8)
    h = np.array(st.history)
    assert h[-1] / h[0] < 0.05
    assert st.dtau_history[1] > st.dtau_history[0]      # SER grows dtau while r falls
    assert st.refreshes == [0]


@pytest.mark.parametrize("name,order", [("esdirk2", 2), ("esdirk3", 3), ("esdirk4", 4)])
def test_esdirk_tableau_order_and_l_stability(name, order):
    A = S.esdirk_tableau(name)
    b, c = A[-1], A.sum(axis=1)
    assert A[0, 0] == 0.0 and np.all(np.diag(A)[1:] == A[1, 1])
    assert abs(b.sum() - 1) < 1e-15 and abs(b @ c - 0.5) < 1e-15
    if order >= 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-14 and abs(b @ (A @ c) - 1 / 6) < 1e-14
    else:
        assert abs(b @ c ** 2 - 1 / 3) > 1e-3
    # the four fourth-order conditions (Butcher trees of order 4)
    o4 = [b @ c ** 3 - 1 / 4, b @ (c * (A @ c)) - 1 / 8, b @ (A @ c ** 2) - 1 / 12, b @ (A @ (A @ c)) - 1 / 24]
    if order >= 4:
        assert np.max(np.abs(o4)) < 1e-14, o4
    else:
        assert np.max(np.abs(o4)) > 1e-4
    # stability function R(z) = 1 + z b^T (I - zA)^{-1} 1 -> 0 as z -> -inf (L-stable, stiffly accurate)
    z = -1e8
    Rz = 1 + z * b @ np.linalg.solve(np.eye(len(b)) - z * A, np.ones(len(b)))
    assert abs(Rz) < 1e-6


def _newton_stage(lev, q, c_mass, src, tol=1e-12):
    """Exact stage solve by Newton's method with the dense complex-step global Jacobian."""
    n = q.size
    for _ in range(20):
        F = lev.stage_residual(q, c_mass, src)
        if np.linalg.norm(F) < tol * 1e3:
            break
        J = np.zeros((n, n))
        for k in range(n):
            qc = q.astype(complex).ravel()
            qc[k] += 1e-30j
            J[:, k] = lev.stage_residual(qc.reshape(q.shape), c_mass, src).imag.ravel() / 1e-30
        q = q - np.linalg.solve(J, F.ravel()).reshape(q.shape)
    return q


@pytest.mark.slow
@pytest.mark.parametrize("name,order", [("esdirk2", 2), ("esdirk3", 3), ("esdirk4", 4)])
def test_esdirk_driver_temporal_order(name, order):
    """Self-convergence in dt of the ESDIRK source construction (eq. (26)) with exact stage solves."""
    mesh = W.periodic_quad_mesh(2, 10.0)
    vs = W.VortexSpec(length=10.0, ma_inf=0.3)
    lev = FRLevel(mesh, 1, GAS)
    A = S.esdirk_tableau(name)
    om = A[1, 1]
    q0 = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    T_end = 0.4
    sols = []
    for nsteps in (4, 8, 16):
        dt = T_end / nsteps
        q = q0.copy()
        for _ in range(nsteps):
            qc_n = G.conservative(q, GAS)
            Rs = [lev.residual(q)]
            qi = q
            for i in range(1, A.shape[0]):
                src = (qc_n + dt * sum(A[i, j] * Rs[j] for j in range(i))) / (om * dt)
                qi = _newton_stage(lev, qi, 1 / (om * dt), src)
                Rs.append(lev.residual(qi))
            q = qi
        sols.append(q)
    e1 = np.linalg.norm(sols[0] - sols[1])
    e2 = np.linalg.norm(sols[1] - sols[2])
    rate = math.log2(e1 / e2)
    # steps of T/4 .. T/16 are pre-asymptotic for the fourth-order scheme (measured 4.34); the band
    # still separates it from third and fifth order
    assert abs(rate - order) < (0.4 if order == 4 else 0.2), rate


def _level_jacobian(level, x, c_mass):
    """Dense dF/dq of a whole level (every element, the neighbours included) by complex step."""
    n = x.size
    A = np.zeros((n, n))
    for k in range(n):
        z = x.astype(complex).ravel()
        z[k] += 1e-30j
        A[:, k] = level.stage_residual(z.reshape(x.shape), c_mass).imag.ravel() / 1e-30
    return A


@pytest.mark.parametrize("Pf,Pc", [(2, 1), (3, 1)])
def test_two_level_fas_correction_is_linear_coarse_solve(Pf, Pc):
    """Sec. 3 with two levels, no fine sweeps and the coarse level solved to convergence: the FAS
    correction added to the fine state, I(q^a_1 - q^b_1), must be I A_c^{-1} P d for a small
    defect d = S_0 - F_0(q), with A_c the Jacobian of the coarse residual at the restricted state
    P q (here a dense complex-step Jacobian of the whole coarse level). The defect is made small
    by the source so that the problem is linear to ~1e-8; Ma 0.3 with a large mass term lets
    element Jacobi converge on the coarse level in 60 sweeps. A sign error on P d, a missing or
    wrong restriction of the state or the defect, or a wrong prolongation fails it; the test also
    shows that A_c at a different coarse state moves the correction by far more than the bound."""
    mesh = W.periodic_quad_mesh(3, 10.0, jitter=0.1, seed=5)
    vs = W.VortexSpec(length=10.0, ma_inf=0.3)
    cm = 10.0
    sol = S.PMGSolver(mesh, GAS, S.PMGOptions(p_levels=(Pf, Pc), n_smooth=(0, 60), dtau_init=1e8))
    lf, lc = sol.levels
    q = vs.state(lf.geo.xy[..., 0], lf.geo.xy[..., 1])
    rng = np.random.default_rng(11)
    src = -lf.stage_residual(q, cm) + 1e-6 * rng.standard_normal(q.shape) * np.abs(lf.residual(q)).max(axis=(0, 1))
    sol.c_mass, sol.src, sol.dtau = cm, src, 1e8
    sol.refresh_now = True
    q1 = sol.vcycle(0, q, None)
    d = -lf.stage_residual(q, cm, src)
    qb = S.restrict(q, Pf, Pc)
    Pd = S.restrict(d, Pf, Pc)
    C = np.linalg.solve(_level_jacobian(lc, qb, cm), Pd.ravel()).reshape(qb.shape)
    want = S.prolong(C, Pc, Pf)
    den = np.linalg.norm(want.reshape(-1, 4), axis=0)
    err = np.linalg.norm((q1 - q - want).reshape(-1, 4), axis=0) / den
    assert np.all(err < 1e-6), err
    # power: the same correction with the coarse Jacobian taken at the element-mean velocity
    qw = qb.copy()
    qw[..., 1:3] = qb[..., 1:3].mean(axis=1, keepdims=True)
    Cw = np.linalg.solve(_level_jacobian(lc, qw, cm), Pd.ravel()).reshape(qb.shape)
    moved = np.linalg.norm((S.prolong(Cw, Pc, Pf) - want).reshape(-1, 4), axis=0) / den
    assert np.all(moved > 100 * 1e-6), moved


@pytest.mark.slow
def test_ser_floor_keeps_dtau_at_or_above_its_start():
    """The SER floor (ser_floor, a reading: eq. (31) states no lower bound) on the stage of the
    stage-guess test below that jumps: without it dtau falls below dtau_init after the jump, with
    it every dtau of the history stays at or above dtau_init, and the first V-cycles, before any
    reduction, are the same."""
    vs = W.VortexSpec(length=20.0, ma_inf=0.005)
    mesh = W.periodic_quad_mesh(8, 20.0)
    tab = S.esdirk_tableau("esdirk2")

    def solver(nvc, floor):
        return S.PMGSolver(mesh, GAS, S.PMGOptions(p_levels=(2, 1, 0), n_smooth=(5, 10, 20), tol=1e-4,
                                                   max_vcycles=nvc, ser_floor=floor), q_inf=vs.freestream())

    sol = solver(60, False)
    lev = sol.levels[0]
    q1, _ = sol.esdirk_step(vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1]), 0.2, tab, stage_guess="previous")
    _, st_free = solver(8, False).esdirk_step(q1, 0.2, tab, stage_guess="previous")
    _, st_floor = solver(8, True).esdirk_step(q1, 0.2, tab, stage_guess="previous")
    d0 = st_free[0].dtau_history[0]
    assert min(st_free[0].dtau_history) < 0.5 * d0
    assert min(st_floor[0].dtau_history) >= d0
    assert st_floor[0].history[:2] == st_free[0].history[:2]


@pytest.mark.slow
def test_stage_guess_predictor_converges_after_first_step():
    """The reading of the stage's initial guess (Sec. 2.4 states none), in the Sec. 4.1 setting
    (vortex on the periodic [-10, 10]^2 square at Ma 0.005, dtau 0.01 -> 10 by eq. (31), blocks
    rebuilt every 10 V-cycles, tolerance 1e-4) on an 8 x 8 mesh at P{2-1-0}, ESDIRK2 with
    dt = 0.2: once a step has been solved, a stage started from the previous stage value begins
    near its solution, so the element-Jacobi sweeps of its first V-cycle raise the relative
    residual by two orders of magnitude and SER collapses dtau; started from the explicit
    predictor the relative residual only falls and both stages of the second step reach the
    tolerance within 40 V-cycles (measured: 26 and 31)."""
    vs = W.VortexSpec(length=20.0, ma_inf=0.005)
    mesh = W.periodic_quad_mesh(8, 20.0)
    tab = S.esdirk_tableau("esdirk2")

    def solver(nvc):
        return S.PMGSolver(mesh, GAS, S.PMGOptions(p_levels=(2, 1, 0), n_smooth=(5, 10, 20), tol=1e-4,
                                                   max_vcycles=nvc), q_inf=vs.freestream())

    sol = solver(60)
    lev = sol.levels[0]
    q1, st0 = sol.esdirk_step(vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1]), 0.2, tab, stage_guess="previous")
    assert all(s.converged for s in st0)
    _, st_prev = solver(3).esdirk_step(q1, 0.2, tab, stage_guess="previous")
    assert max(st_prev[0].history) / st_prev[0].history[0] > 50.0
    _, st_pred = solver(40).esdirk_step(q1, 0.2, tab, stage_guess="predictor")
    for s in st_pred:
        assert s.converged, s.history
        assert max(s.history) <= 1.0 * s.history[0]


def test_vcycle_without_rebuild_does_not_depend_on_dtau():
    """Delta tau enters the V-cycle only through the element blocks (eqs. (28)-(30)): between block
    rebuilds the same blocks and state give the same V-cycle for any Delta tau. The stage solve's
    lookahead on the GPU (the V-cycle after the one in flight enqueued before the SER law has set
    Delta tau from the in-flight norm) is exact because of this."""
    mesh, vs = _vortex(n=3, P=2)
    sol = S.PMGSolver(mesh, GAS, S.PMGOptions(p_levels=(2, 1, 0), n_smooth=(2, 3, 4)), q_inf=vs.freestream())
    q = vs.state(sol.levels[0].geo.xy[..., 0], sol.levels[0].geo.xy[..., 1])
    sol.dtau = 0.05
    sol.refresh_now = True                   # blocks of every level, as at a rebuild
    sol.build_D(0, q)
    q1 = sol.vcycle(0, q, None)
    sol.refresh_now = False
    outs = []
    for dtau in (1e-3, 0.05, 7.0):
        sol.dtau = dtau
        outs.append(sol.vcycle(0, q1, None))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    sol.dtau = 7.0                           # a rebuild at another Delta tau does change the cycle
    sol.refresh_now = True
    sol.build_D(0, q1)
    assert not np.array_equal(sol.vcycle(0, q1, None), outs[1])
