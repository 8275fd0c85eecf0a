"""FR/CPR spatial residual with the preconditioned common flux (Sec. 2.3) and the
ESDIRK stage residual (Sec. 2.4, eq. (26)).

R = -div f is evaluated in the differential FR form of eq. (20): the divergence of
the Lagrange interpolant of the transformed flux plus the correction field built
from 1-D correction polynomials along each tensor line,

  R_ij = -(1/|J_ij|) [ sum_k D_ik F~_kj + g_L'(xi_i)(F^_L,j - F~_L,j) + g_R'(xi_i)(F^_R,j - F~_R,j)
                       + sum_k D_jk G~_ik + g_L'(eta_j)(G^_B,i - G~_B,i) + g_R'(eta_j)(G^_T,i - G~_T,i) ],

where F~_L,j = sum_k l_k(-1) F~_kj is the interpolated local flux at the face and
F^ = |S| f_com is the common flux of eq. (21) in the +xi direction.

Boundary states (the paper does not state them): periodic faces are identified;
a slip wall uses the ghost (p, u - 2(u.n)n, T); a no-slip adiabatic wall the ghost
(p, -u, -v, T); a far-field face uses the free stream q_inf; all pass through the same
common flux.

With a viscosity mu > 0 the BR2 viscous terms of ``oracle.viscous`` are subtracted from
the transformed fluxes and the common fluxes (R = -div(f_inv - f_vis)).
"""
from __future__ import annotations

import numpy as np

from . import gas as G
from .basis import Ops1D
from .geometry import QuadGeometry
from .viscous import BR2

BC_SLIP_WALL = -1
BC_FAR_FIELD = -2
BC_NOSLIP_WALL = -3


class FRLevel:
    """One P-level of a 2-D quad mesh."""

    def __init__(self, mesh, P: int, gas: G.Gas, q_inf=None):
        assert mesh.dim == 2
        self.mesh = mesh
        self.P = P
        self.gas = gas
        self.ops = Ops1D(P)
        self.geo = QuadGeometry(mesh, P)
        self.n1 = P + 1
        self.nv = 4
        self.npts = self.n1 * self.n1
        self.n = self.nv * self.npts
        self.ne = mesh.n_elements
        self.q_inf = None if q_inf is None else np.asarray(q_inf, float)
        self.br2 = BR2(self) if gas.mu > 0.0 else None

    # ---- face traces -------------------------------------------------------------
    def traces(self, q):
        """Own-side states at the flux points, [Ne, 4, P+1, Nv] (extrapolation along lines)."""
        o = self.ops
        q4 = q.reshape(self.ne, self.n1, self.n1, self.nv)  # [e, j, i, v]
        tl = np.einsum("k,ejkv->ejv", o.lm, q4)
        tr = np.einsum("k,ejkv->ejv", o.lp, q4)
        tb = np.einsum("k,ekiv->eiv", o.lm, q4)
        tt = np.einsum("k,ekiv->eiv", o.lp, q4)
        return np.stack([tl, tr, tb, tt], axis=1)

    def neighbour_face_values(self, x):
        """For per-face values x [Ne, 4, P+1, ...] of every element, the neighbour's values on
        the shared face seen from each (element, face), in this face's point order (zero on
        boundary faces)."""
        m = self.mesh
        out = np.zeros_like(x)
        for f in range(4):
            nb = m.face_nbr[:, f]
            inner = nb >= 0
            idx = np.where(inner, nb, 0)
            tr = x[idx, m.face_nbr_face[:, f]]
            flip = (m.face_orient[:, f] == 1).reshape((-1,) + (1,) * (tr.ndim - 1))
            tr = np.where(flip, tr[:, ::-1], tr)
            out[:, f] = np.where(inner.reshape((-1,) + (1,) * (tr.ndim - 1)), tr, 0.0)
        return out

    def outside_states(self, own, nbr_tr):
        """State across each face: the neighbour's trace, or a boundary ghost."""
        m = self.mesh
        out = self.neighbour_face_values(nbr_tr).astype(np.result_type(own, nbr_tr))
        for f in range(4):
            nb = m.face_nbr[:, f]
            wall = nb == BC_SLIP_WALL
            if np.any(wall):
                nvec = self.geo.fvec[:, f]
                nunit = nvec / np.sqrt(np.sum(nvec * nvec, axis=-1))[..., None]
                u = own[:, f, :, 1:3]
                un = np.sum(u * nunit, axis=-1)
                ghost = own[:, f].copy()
                ghost[..., 1:3] = u - 2.0 * un[..., None] * nunit
                out[:, f] = np.where(wall[:, None, None], ghost, out[:, f])
            noslip = nb == BC_NOSLIP_WALL
            if np.any(noslip):
                ghost = own[:, f].copy()
                ghost[..., 1:3] = -own[:, f, :, 1:3]
                out[:, f] = np.where(noslip[:, None, None], ghost, out[:, f])
            far = nb == BC_FAR_FIELD
            if np.any(far):
                out[:, f] = np.where(far[:, None, None], self.q_inf, out[:, f])
        return out

    def viscous_terms(self, q, q_nbr, own, out):
        """BR2 transformed viscous fluxes at the solution points and common viscous fluxes at
        the faces (``oracle.viscous``); the neighbours' gradients come from q_nbr (default q)."""
        br2, m, g = self.br2, self.mesh, self.geo
        qn = q if q_nbr is None else q_nbr
        qcom = 0.5 * (own + out)
        # the outside side's grad q + r on each interior face: the neighbour's local gradient
        # and its lifting of that face, whose jump q_com - q+ uses this element's trace
        gl_n = self.neighbour_face_values(br2.face_local_gradients(qn))
        n_vec = self.neighbour_face_values(g.fvec)
        n_lam = self.neighbour_face_values(br2.lam)
        out_grad = gl_n + br2.penalty * (qcom - out)[..., None] * n_vec[:, :, :, None, :] * n_lam[..., None, None]
        one_sided = m.face_nbr < 0
        return br2.terms(q, own, out, out_grad, one_sided, m.face_nbr == BC_NOSLIP_WALL, m.face_nbr == BC_FAR_FIELD)

    # ---- residual ----------------------------------------------------------------
    def residual(self, q, q_nbr=None, nbr_faces=None):
        """R(q) = -div f at the solution points, [Ne, Np, Nv].

        ``q_nbr`` (default q) is the state the neighbours' face traces are taken from;
        the Jacobian module passes the unperturbed state there so that only the
        element's own unknowns move. With ``nbr_faces`` (a tuple of face indices) only
        those faces of every element see q_nbr; the others see the neighbours' traces of q
        (inviscid only), so that the response of element e measures its coupling to the one
        neighbour across each listed face.
        """
        o, g = self.ops, self.geo
        ne, n1, nv = self.ne, self.n1, self.nv
        own = self.traces(q)
        nbr_tr = own if q_nbr is None else self.traces(q_nbr)
        out = self.outside_states(own, nbr_tr)
        if nbr_faces is not None:
            if self.br2 is not None:
                raise ValueError("per-face neighbour states are defined for inviscid levels only")
            keep = np.zeros(4, bool)
            keep[list(nbr_faces)] = True
            out = np.where(keep[None, :, None, None], out, self.outside_states(own, own))
        fv = g.fvec
        fh = [G.common_flux(out[:, 0], own[:, 0], fv[:, 0], self.gas),
              G.common_flux(own[:, 1], out[:, 1], fv[:, 1], self.gas),
              G.common_flux(out[:, 2], own[:, 2], fv[:, 2], self.gas),
              G.common_flux(own[:, 3], out[:, 3], fv[:, 3], self.gas)]
        ft = G.normal_flux(q, g.S_sp, self.gas).reshape(ne, n1, n1, nv)  # [e, j, i, v]
        gt = G.normal_flux(q, g.T_sp, self.gas).reshape(ne, n1, n1, nv)
        if self.br2 is not None:            # total flux f_inv - f_vis
            fvt, gvt, fhv = self.viscous_terms(q, q_nbr, own, out)
            ft = ft - fvt
            gt = gt - gvt
            fh = [fh[f] - fhv[:, f] for f in range(4)]
        fl = np.einsum("k,ejkv->ejv", o.lm, ft)
        fr = np.einsum("k,ejkv->ejv", o.lp, ft)
        gb = np.einsum("k,ekiv->eiv", o.lm, gt)
        gtt = np.einsum("k,ekiv->eiv", o.lp, gt)
        div = np.einsum("ik,ejkv->ejiv", o.D, ft)
        div = div + o.gL[None, None, :, None] * (fh[0] - fl)[:, :, None, :]
        div = div + o.gR[None, None, :, None] * (fh[1] - fr)[:, :, None, :]
        div = div + np.einsum("jk,ekiv->ejiv", o.D, gt)
        div = div + o.gL[None, :, None, None] * (fh[2] - gb)[:, None, :, :]
        div = div + o.gR[None, :, None, None] * (fh[3] - gtt)[:, None, :, :]
        return -div.reshape(ne, self.npts, nv) / g.jac[..., None]

    def stage_residual(self, q, c_mass=0.0, src=None, S=None, q_nbr=None):
        """F(q) - S with F = R(q) - c_mass q_c(q) + src (eq. (26); c_mass = 1/(omega dt),
        0 for a steady problem, where F = R)."""
        F = self.residual(q, q_nbr)
        if c_mass != 0.0:
            F = F - c_mass * G.conservative(q, self.gas)
        if src is not None:
            F = F + src
        if S is not None:
            F = F - S
        return F
