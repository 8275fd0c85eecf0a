"""Pins of the oracle's FR/CPR residual: free-stream preservation, discrete conservation,
and the truncation error against the closed-form vortex (Sec. 4.1, eq. (46))."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle.fr import FRLevel

GAS = G.Gas(eps_mode="local")


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_freestream_preserved_on_jittered_mesh(P):
    mesh = W.periodic_quad_mesh(6, 10.0, jitter=0.1, seed=7)
    vs = W.VortexSpec(length=10.0)
    lev = FRLevel(mesh, P, GAS)
    q = np.broadcast_to(vs.freestream(), (lev.ne, lev.npts, 4)).copy()
    R = lev.residual(q)
    speed = np.hypot(*vs.u_inf)
    # every term of R is a flux divided by an element size: p_inf |V_inf| max(|S|/|J|)
    inv_h = np.max(np.linalg.norm(lev.geo.S_sp, axis=-1) / lev.geo.jac)
    scale = vs.p_inf * speed * inv_h
    assert np.max(np.abs(R[..., :3])) / scale < 1e-13
    # Energy: the preconditioned dissipation multiplies the rounding of the pressure traces
    # by Gamma's (Theta H - 1) ~ H/U_r^2 = H/(eps c)^2, i.e. by 1/eps^2 relative to the
    # energy flux rho H |V| (eqs. (9), (10), (21)); eps = Ma here.
    h_inf = GAS.cp * vs.t_inf + 0.5 * speed ** 2
    escale = vs.rho_inf * h_inf * speed * inv_h
    assert np.max(np.abs(R[..., 3])) / escale < 1e-13 / vs.ma_inf ** 2


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_discrete_conservation(P):
    """sum_e sum_p w_p |J| R = 0: interior common fluxes cancel pairwise, so the FR/DG
    residual conserves every conservative component on a periodic mesh."""
    mesh, vs = W.periodic_quad_mesh(5, 10.0, jitter=0.1, seed=11), W.VortexSpec(length=10.0)
    lev = FRLevel(mesh, P, GAS)
    q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    R = lev.residual(q)
    w = np.outer(lev.ops.w, lev.ops.w).ravel()       # p = i + (P+1) j, weight w_i w_j
    tot = np.einsum("p,ep,epv->v", w, lev.geo.jac, R)
    # the sum cancels face fluxes of size |f(q_inf)| |S| pairwise: rounding is relative to those
    perimeter = np.einsum("k,efk->", lev.ops.w, np.linalg.norm(lev.geo.fvec, axis=-1))
    speed = np.hypot(*vs.u_inf)
    h_inf = GAS.cp * vs.t_inf + 0.5 * speed ** 2
    fscale = np.array([vs.rho_inf * speed, vs.p_inf, vs.p_inf, vs.rho_inf * h_inf * speed])
    assert np.all(np.abs(tot) <= 1e-13 * fscale * perimeter), tot / (fscale * perimeter)


def _exact_dqc_dt(vs, xy, h=1e-4):
    qp = G.conservative(vs.state(xy[..., 0], xy[..., 1], h), GAS)
    qm = G.conservative(vs.state(xy[..., 0], xy[..., 1], -h), GAS)
    return (qp - qm) / (2 * h)


@pytest.mark.parametrize("P", [2, 3])
def test_truncation_error_order(P):
    """R(q_exact) -> d q_c/dt of the translating vortex at rate >= P (pointwise FR truncation)."""
    vs = W.VortexSpec(length=20.0)
    errs = []
    for n in (6, 12, 24):
        lev = FRLevel(W.periodic_quad_mesh(n, 20.0, jitter=0.0), P, GAS)
        xy = lev.geo.xy
        R = lev.residual(vs.state(xy[..., 0], xy[..., 1]))
        ref = _exact_dqc_dt(vs, xy)
        w = np.outer(lev.ops.w, lev.ops.w).ravel()
        e = np.sqrt(np.einsum("p,ep,epv->v", w, lev.geo.jac, (R - ref) ** 2))
        errs.append(e[1:3].max())                     # momentum, where the vortex lives
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= P - 0.3, (errs, rates)
