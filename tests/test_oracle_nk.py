"""Oracle pins for the Newton-Krylov stage solve (the V-cycle as a preconditioner of flexible
GMRES on the pseudo-transient Newton system of eqs. (27)-(28) with the whole Jacobian): with as
many Krylov directions as unknowns GMRES is exact, so one Newton step must equal the dense solve
of (Gamma/dtau - dF/dq) delta = F(q) with dF/dq by complex step, with and without the
preconditioner; and the preconditioner is linear to first order in its scale."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS

VS = W.VortexSpec(length=10.0, ma_inf=0.3)
GAS = OG.Gas(gamma=VS.gamma, rgas=VS.rgas, eps_mode="local")


def _setup(dtau):
    mesh = W.periodic_quad_mesh(2, 10.0, jitter=0.1)
    opts = OS.PMGOptions(p_levels=(1, 0), n_smooth=(2, 4), dtau_init=dtau, dtau_max=dtau, tol=1e-30)
    sol = OS.PMGSolver(mesh, GAS, opts, q_inf=VS.freestream())
    lev = sol.levels[0]
    q = VS.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    return sol, lev, q


def _dense_newton_step(sol, lev, q, c_mass, src, dtau):
    n = q.size
    J = np.zeros((n, n))
    for k in range(n):
        qc = q.astype(complex).ravel()
        qc[k] += 1e-30j
        J[:, k] = lev.stage_residual(qc.reshape(q.shape), c_mass, src).imag.ravel() / 1e-30
    gam = OG.preconditioner(q, GAS)
    Gd = np.zeros((n, n))
    nv = q.shape[-1]
    for e in range(q.shape[0]):
        for p in range(q.shape[1]):
            i0 = (e * q.shape[1] + p) * nv
            Gd[i0:i0 + nv, i0:i0 + nv] = gam[e, p]
    A = Gd / dtau - J
    F0 = lev.stage_residual(q, c_mass, src).ravel()
    return np.linalg.solve(A, F0).reshape(q.shape)


@pytest.mark.parametrize("precondition", [False, True])
def test_one_newton_step_is_the_dense_solve(precondition):
    dtau = 0.3
    sol, lev, q = _setup(dtau)
    c_mass = 1.0 / (0.29 * 0.05)
    src = OG.conservative(q, GAS) * c_mass * 1.001        # a source that makes F(q) != 0 everywhere
    ref = _dense_newton_step(sol, lev, q, c_mass, src, dtau)
    q1, st = sol.nk_stage_solve(q, c_mass, src, krylov_dim=q.size, eta=1e-13, max_newton=1,
                                precondition=precondition, fd_rel=1e-7, pc_rel=1e-7)
    delta = q1 - q
    err = np.max(np.abs(delta - ref), axis=(0, 1)) / np.max(np.abs(ref), axis=(0, 1))
    assert st.n_vcycles == 1 and st.krylov <= q.size
    assert np.all(err < 2e-5), err
    if precondition:                  # the V-cycle preconditioner needs far fewer directions
        _, st2 = sol.nk_stage_solve(q, c_mass, src, krylov_dim=q.size, eta=1e-6, max_newton=1,
                                    fd_rel=1e-7, pc_rel=1e-7)
        _, st3 = sol.nk_stage_solve(q, c_mass, src, krylov_dim=q.size, eta=1e-6, max_newton=1,
                                    precondition=False, fd_rel=1e-7, pc_rel=1e-7)
        assert st2.krylov < st3.krylov, (st2.krylov, st3.krylov)


def test_newton_krylov_converges_fast_at_large_dtau():
    """At dtau -> infinity the steps are Newton's: on the second ESDIRK2 stage equation the
    residual falls quadratically."""
    sol, lev, q = _setup(1e8)
    A = OS.esdirk_tableau("esdirk2")
    dt, om = 0.05, A[1, 1]
    src = (OG.conservative(q, GAS) + dt * A[1, 0] * lev.residual(q)) / (om * dt)
    q1, st = sol.nk_stage_solve(q, 1.0 / (om * dt), src, krylov_dim=q.size, eta=1e-12, max_newton=3,
                                fd_rel=1e-7, pc_rel=1e-7)
    h = np.array(st.history) / st.history[0]
    assert h[1] < 1e-2 and h[2] < 10.0 * h[1] ** 2 and h[3] < 10.0 * h[2] ** 2 + 1e-13, h
