"""Viscous fluxes with the second Bassi-Rebay (BR2) common gradient (Sec. 2.1 and Sec. 2.3).

Physical viscous flux (Sec. 2.1), primitive variables (p, u, v, T) and their gradients:
  tau_ij = 2 mu (S_ij - (div u)/3 delta_ij),  S_ij = (du_i/dx_j + du_j/dx_i)/2,
  K_j = -(mu C_p / Pr) dT/dx_j,
  f_vis,j = (0, tau_1j, tau_2j, u_i tau_ij - K_j).
The residual is R = -div(f_inv - f_vis).

Common values on a face (eqs. (22), (23)): q_com = (q- + q+)/2 and
grad q_com = ((grad q- + r-) + (grad q+ + r+))/2, with r+- the BR2 corrections of the gradient
on that face.

Readings (the paper names BR2 and gives eqs. (22)-(23) only):
* Local gradient at a solution point: the chain rule on the solution polynomial,
  grad q = (S dq/dxi + T dq/deta)/|J| with S = (y_eta, -x_eta), T = (-y_xi, x_xi).
* Lifting of face f into its element, at a solution point on the tensor line through flux
  point k of f: r_f = g_f'(xi) (q_com - q_f)_k N_f,k / |J|, the FR correction of the gradient
  "flux" q (N_f,k is the face vector in the +xi / +eta direction whose length is the face
  Jacobian, the same vector that scales the common inviscid flux). It vanishes when the trace is
  continuous.
* Corrected gradient used by the volume viscous flux: grad q + sum over the four faces of r_f.
* r+- on a face: each side's own lifting of that face alone, extrapolated along its line to the
  flux point and multiplied by the BR2 penalty eta; grad q+- there: the local gradients
  extrapolated along the same line.
* Penalty eta (not given): the number of faces of the element, 4 for quadrilaterals, the value
  BR2's stability analysis asks for (``Gas.br2_penalty``). With eta = 1 the discrete compressible
  stress operator is indefinite (one mode grows) for P >= 2; from eta = 2 on it is symmetric and
  negative semi-definite (tested).
* Boundary faces: q_com is the boundary state and the gradient is one-sided,
  grad q_com = grad q- + eta r-, with r- lifting q_com - q-: the far field takes q_com = q_inf;
  at walls q_com is the mean of the trace and its ghost, which is the boundary state itself
  (slip wall: normal velocity removed; no-slip adiabatic wall: ghost (p, -u, -v, T), so
  q_com = (p, 0, 0, T), and the wall-normal component of grad T is removed from grad q_com, so no
  heat crosses the wall). Taking the mean with the far-field ghost instead would make the discrete
  viscous operator unsymmetric (tested).
* The common viscous flux on a face is N . f_vis(q_com, grad q_com); the element's local
  viscous flux at the face is the Lagrange interpolant of its transformed viscous flux, as for
  the inviscid part.
"""
from __future__ import annotations

import numpy as np


def viscous_flux(q, grad, gas):
    """(f_vis,x, f_vis,y), each [..., 4], from states [..., 4] and gradients [..., 4, 2]."""
    u, v = q[..., 1], q[..., 2]
    ux, uy = grad[..., 1, 0], grad[..., 1, 1]
    vx, vy = grad[..., 2, 0], grad[..., 2, 1]
    tx, ty = grad[..., 3, 0], grad[..., 3, 1]
    mu = gas.mu
    div = ux + vy
    txx = 2.0 * mu * (ux - div / 3.0)
    tyy = 2.0 * mu * (vy - div / 3.0)
    txy = mu * (uy + vx)
    k = mu * gas.cp / gas.prandtl
    Kx, Ky = -k * tx, -k * ty
    zero = np.zeros_like(u)
    fx = np.stack([zero, txx, txy, u * txx + v * txy - Kx], axis=-1)
    fy = np.stack([zero, txy, tyy, u * txy + v * tyy - Ky], axis=-1)
    return fx, fy


def line_extrapolate(ops, x, face):
    """Values at the flux points of one face from solution-point values x [Ne, n1, n1, ...]
    (index [e, j, i]) by the Lagrange basis along each tensor line."""
    w = ops.lm if face in (0, 2) else ops.lp
    if face < 2:
        return np.einsum("k,ejk...->ej...", w, x)
    return np.einsum("k,eki...->ei...", w, x)


class BR2:
    """Viscous part of the residual on one FRLevel (the level supplies geometry and operators)."""

    def __init__(self, level):
        self.lev = level
        self.penalty = level.gas.br2_penalty
        g, o, n1 = level.geo, level.ops, level.n1
        ne = level.ne
        jac = g.jac.reshape(ne, n1, n1)                        # [e, j, i]
        # lambda_f,k = sum_m l_m(face) g_f'(x_m) / |J_m| along the line of flux point k
        self.lam = np.zeros((ne, 4, n1))
        self.lam[:, 0] = np.einsum("m,m,ejm->ej", o.lm, o.gL, 1.0 / jac)
        self.lam[:, 1] = np.einsum("m,m,ejm->ej", o.lp, o.gR, 1.0 / jac)
        self.lam[:, 2] = np.einsum("m,m,emi->ei", o.lm, o.gL, 1.0 / jac)
        self.lam[:, 3] = np.einsum("m,m,emi->ei", o.lp, o.gR, 1.0 / jac)

    def local_gradient(self, q):
        """Chain-rule gradient of the solution polynomial at the solution points, [Ne, Np, 4, 2]."""
        lev = self.lev
        o, g, ne, n1 = lev.ops, lev.geo, lev.ne, lev.n1
        q4 = q.reshape(ne, n1, n1, 4)
        dxi = np.einsum("ik,ejkv->ejiv", o.D, q4).reshape(ne, -1, 4)
        deta = np.einsum("jk,ekiv->ejiv", o.D, q4).reshape(ne, -1, 4)
        return (g.S_sp[:, :, None, :] * dxi[..., None] + g.T_sp[:, :, None, :] * deta[..., None]) \
            / g.jac[:, :, None, None]

    def liftings(self, jump):
        """r_f at the solution points for each face, [4, Ne, Np, 4, 2], from the jumps
        (q_com - q_own) at the flux points, jump [Ne, 4, n1, 4]."""
        lev = self.lev
        o, g, ne, n1 = lev.ops, lev.geo, lev.ne, lev.n1
        jac = g.jac.reshape(ne, n1, n1)
        out = np.zeros((4, ne, n1, n1, 4, 2), dtype=jump.dtype)
        for f in range(4):
            jn = jump[:, f, :, :, None] * g.fvec[:, f, :, None, :]      # [e, k, v, d]
            gp = o.gL if f in (0, 2) else o.gR
            if f < 2:       # line j, point i: g'(xi_i) jn[e, j] / |J_ji|
                out[f] = gp[None, None, :, None, None] * jn[:, :, None] / jac[..., None, None]
            else:           # line i, point j: g'(eta_j) jn[e, i] / |J_ji|
                out[f] = gp[None, :, None, None, None] * jn[:, None, :] / jac[..., None, None]
        return out.reshape(4, ne, n1 * n1, 4, 2)

    def face_lifting(self, jump):
        """Each face's lifting extrapolated to its own flux points, (q_com - q_own) N lambda,
        [Ne, 4, n1, 4, 2], with lambda_f,k = sum_m l_m(face) g_f'(x_m) / |J_m| along the line."""
        g = self.lev.geo
        return self.penalty * jump[..., None] * g.fvec[:, :, :, None, :] * self.lam[:, :, :, None, None]

    def face_local_gradients(self, q):
        """Local gradients extrapolated to the flux points of every face, [Ne, 4, n1, 4, 2]."""
        lev = self.lev
        g4 = self.local_gradient(q).reshape(lev.ne, lev.n1, lev.n1, 4, 2)
        return np.stack([line_extrapolate(lev.ops, g4, f) for f in range(4)], axis=1)

    def terms(self, q, own, out, out_grad, one_sided, wall_noslip, far_field):
        """Viscous transformed fluxes at the solution points (F~v, G~v, each [Ne, n1(j), n1(i), 4])
        and common viscous fluxes N . f_vis at the flux points of each face ([Ne, 4, n1, 4]).

        own, out: own traces and outside states [Ne, 4, n1, 4]; out_grad: the outside side's
        (grad q + r) at each flux point [Ne, 4, n1, 4, 2] (ignored on one-sided faces);
        one_sided, wall_noslip, far_field: [Ne, 4] masks of boundary faces, of no-slip adiabatic
        walls and of far-field faces (where q_com is the free stream itself).
        """
        lev = self.lev
        g, ne, n1, gas = lev.geo, lev.ne, lev.n1, lev.gas
        qcom = np.where(far_field[:, :, None, None], out, 0.5 * (own + out))
        jump = qcom - own
        grad = self.local_gradient(q)
        gcor = grad + self.liftings(jump).sum(axis=0)
        fx, fy = viscous_flux(q, gcor, gas)
        Sx, Sy = g.S_sp[..., 0:1], g.S_sp[..., 1:2]
        Tx, Ty = g.T_sp[..., 0:1], g.T_sp[..., 1:2]
        fv_t = (Sx * fx + Sy * fy).reshape(ne, n1, n1, 4)
        gv_t = (Tx * fx + Ty * fy).reshape(ne, n1, n1, 4)
        own_side = self.face_local_gradients(q) + self.face_lifting(jump)
        os_mask = one_sided[:, :, None, None, None]
        gcom = np.where(os_mask, own_side, 0.5 * (own_side + np.where(os_mask, 0.0, out_grad)))
        nvec = g.fvec                                                     # [e, f, k, 2]
        if np.any(wall_noslip):
            nunit = nvec / np.sqrt(np.sum(nvec * nvec, axis=-1))[..., None]
            gt = gcom[..., 3, :]
            gt_wall = gt - np.sum(gt * nunit, axis=-1)[..., None] * nunit
            gcom = gcom.copy()
            gcom[..., 3, :] = np.where(wall_noslip[:, :, None, None], gt_wall, gt)
        cx, cy = viscous_flux(qcom, gcom, gas)
        fhat = nvec[..., 0:1] * cx + nvec[..., 1:2] * cy
        return fv_t, gv_t, fhat
