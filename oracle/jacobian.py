"""Element-diagonal blocks of the pseudo-transient linearisation (Sec. 2.4).

A = Gamma/dtau + M/(omega dt) - dR/dq_p (eq. (28)) is -dF/dq_p + Gamma/dtau for the stage
residual F of eq. (26); the element-Jacobi smoother keeps only its block diagonal D
(eq. (30)): the derivative of element e's residual with respect to element e's own
unknowns, the neighbours held fixed.

Reading: D is the exact block of that Jacobian, including the dependence of the
common flux's averaged state, eigenvalues and preconditioner on the unknowns (the
paper does not say how its Jacobian is formed). It is computed here column by
column with the complex step, dF/dq_c ~= Im F(q + i h e_c) / h, which is exact to
rounding because no difference is taken. Forcing terms S and sources do not depend
on q and drop out.
"""
from __future__ import annotations

import numpy as np

from . import gas as G

H_STEP = 1e-30


def element_dFdq(level, q, c_mass=0.0):
    """dF_e/dq_e for every element, [Ne, n, n] with index p*Nv + v."""
    ne, npts, nv = q.shape
    n = npts * nv
    out = np.zeros((ne, n, n))
    qr = np.asarray(q, float)
    for c in range(n):
        p, v = divmod(c, nv)
        qc = qr.astype(complex)
        qc[:, p, v] += 1j * H_STEP
        F = level.stage_residual(qc, c_mass=c_mass, q_nbr=qr)
        out[:, :, c] = F.imag.reshape(ne, n) / H_STEP
    return out


def pseudo_time_blocks(level, q, dtau):
    """Block-diagonal Gamma(q)/dtau at every solution point, [Ne, n, n]."""
    ne, npts, nv = q.shape
    gam = G.preconditioner(q, level.gas)          # [Ne, Np, Nv, Nv], pointwise eps
    out = np.zeros((ne, npts * nv, npts * nv))
    for p in range(npts):
        out[:, p * nv:(p + 1) * nv, p * nv:(p + 1) * nv] = gam[:, p] / dtau
    return out


def element_blocks(level, q, dtau, c_mass=0.0):
    """D_e = Gamma/dtau - dF_e/dq_e (eqs. (28), (30))."""
    return pseudo_time_blocks(level, q, dtau) - element_dFdq(level, q, c_mass)
