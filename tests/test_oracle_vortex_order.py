"""Spatial order of accuracy of the oracle's FR/CPR residual against the isentropic vortex's closed
form (Sec. 4.1, eq. (46)): the velocity error falls at the rate P + 1 (the trend of Table 2).

The semi-discrete system dq_c/dt = R(q) is advanced with the classical fourth-order Runge-Kutta
method and a step small enough that the temporal error is far below the spatial one, on the
paper's periodic [-10, 10]^2 domain, and the solution is compared with the vortex translated by
the free stream. Explicit time steps must follow the sound speed, so the free-stream Mach number
is 0.5 here (referred to |V_inf| = sqrt(2), as everywhere in this repository) instead of the
paper's 0.005, which would take a hundred times as many steps; the residual takes the same code
path (eps = min(1, Ma) of eq. (11) with the cut-off off, Ma < 1 everywhere). The error is the
|J|-weighted Gauss-quadrature L2 norm over the solution points, per primitive variable.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle.fr import FRLevel

GAS = G.Gas(eps_mode="local")


def _primitive(qc):
    """(rho, rho u, rho v, rho E) -> (p, u, v, T) for the ideal gas with R = GAS.rgas."""
    rho = qc[..., 0]
    u = qc[..., 1:-1] / rho[..., None]
    p = (GAS.gamma - 1.0) * (qc[..., -1] - 0.5 * rho * np.sum(u * u, axis=-1))
    return np.concatenate([p[..., None], u, (p / (rho * GAS.rgas))[..., None]], axis=-1)


def _vortex_error(n, P, t_end, cfl=0.25):
    vs = W.VortexSpec(length=20.0, ma_inf=0.5)
    lev = FRLevel(W.periodic_quad_mesh(n, 20.0), P, GAS)
    x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
    h = 20.0 / n
    speed = vs.c_inf + math.sqrt(2.0) + 1.4          # sound + free stream + vortex peak speed
    steps = int(math.ceil(t_end / (cfl * h / ((2 * P + 1) * speed))))
    dt = t_end / steps
    qc = G.conservative(vs.state(x, y), GAS)

    def rhs(u):
        return lev.residual(_primitive(u))

    for _ in range(steps):
        k1 = rhs(qc)
        k2 = rhs(qc + 0.5 * dt * k1)
        k3 = rhs(qc + 0.5 * dt * k2)
        k4 = rhs(qc + dt * k3)
        qc = qc + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    err = _primitive(qc) - vs.state(x, y, t=t_end)
    w = lev.geo.jac.reshape(lev.ne, -1) * np.outer(lev.ops.w, lev.ops.w).ravel()[None, :]
    return np.sqrt(np.sum(w[..., None] * err ** 2, axis=(0, 1)) / np.sum(w))


@pytest.mark.slow
@pytest.mark.parametrize("P,meshes,t_end", [(2, (16, 32), 1.0), (3, (12, 24), 0.5)])
def test_vortex_velocity_order_is_p_plus_one(P, meshes, t_end):
    """Measured on these meshes: P2 (16 -> 32, t = 1) u 3.07, v 3.11; P3 (12 -> 24, t = 0.5)
    u 4.05, v 4.05. A correction function or derivative operator of lower accuracy, a
    wrong face normal or a wrong sign in the common flux's dissipation brings the rate down or
    makes the run blow up."""
    e0, e1 = (_vortex_error(n, P, t_end) for n in meshes)
    rate = np.log(e0 / e1) / np.log(meshes[1] / meshes[0])
    assert np.all(np.isfinite(rate))
    assert np.all(rate[1:3] >= P + 1 - 0.3), rate
