"""FR/CPR spatial residual on hexahedra with the preconditioned common flux (Sec. 2.3 in three
dimensions) and the ESDIRK stage residual (Sec. 2.4, eq. (26)).

The residual is the three-dimensional form of eq. (20): along each of the three tensor lines the
derivative of the Lagrange interpolant of the transformed flux plus the 1-D correction field,

  R_ijk = -(1/|J|) [ sum_m D_im F~_mjk + g_L'(xi_i)(F^ - F~)_0,jk + g_R'(xi_i)(F^ - F~)_1,jk
                   + (the same along eta with faces 2, 3 and along zeta with faces 4, 5) ],

with F~ = f . (J grad xi^d) the transformed flux of direction d, (F~)_f its interpolant on face f
and F^ = |S| f_com of eq. (21) in the +xi^d direction. Primitive variables (p, u, v, w, T).
Boundaries as in two dimensions: a slip wall uses the mirrored ghost (p, u - 2(u.n)n, T), a
far-field face the free stream.
"""
from __future__ import annotations

import numpy as np

from . import gas as G
from .basis import Ops1D
from .geometry3d import HexGeometry

BC_SLIP_WALL = -1
BC_FAR_FIELD = -2


def orient_map(orient: int, n1: int) -> np.ndarray:
    """Index k1' + n1 k2' of the neighbour's face point met by point k1 + n1 k2, for the
    orientation code of the mesh (swap the pair if bit 0, reverse the first index if bit 1,
    the second if bit 2)."""
    out = np.zeros(n1 * n1, int)
    for k2 in range(n1):
        for k1 in range(n1):
            a, b = (k2, k1) if orient & 1 else (k1, k2)
            if orient & 2:
                a = n1 - 1 - a
            if orient & 4:
                b = n1 - 1 - b
            out[k1 + n1 * k2] = a + n1 * b
    return out


class FRLevel3:
    """One P-level of a 3-D hexahedral mesh."""

    def __init__(self, mesh, P: int, gas: G.Gas, q_inf=None):
        assert mesh.dim == 3
        self.mesh = mesh
        self.P = P
        self.gas = gas
        self.ops = Ops1D(P)
        self.geo = HexGeometry(mesh, P)
        self.n1 = P + 1
        self.nv = 5
        self.npts = self.n1 ** 3
        self.nf = self.n1 ** 2
        self.n = self.nv * self.npts
        self.ne = mesh.n_elements
        self.q_inf = None if q_inf is None else np.asarray(q_inf, float)
        self._omaps = np.stack([orient_map(o, self.n1) for o in range(8)])
        if gas.mu > 0.0:
            raise NotImplementedError("viscous terms are two-dimensional only")

    # ---- face values -------------------------------------------------------------
    def face_interp(self, x, f):
        """Interpolant of point values x [Ne, Np, ...] on face f: [Ne, (P+1)^2, ...] in the face's
        point order k1 + (P+1) k2."""
        o, n1 = self.ops, self.n1
        w = o.lm if f % 2 == 0 else o.lp
        x5 = x.reshape((x.shape[0], n1, n1, n1) + x.shape[2:])          # [e, k, j, i, ...]
        if f < 2:
            y = np.einsum("i,ekji...->ekj...", w, x5)                    # (k2 = k, k1 = j)
        elif f < 4:
            y = np.einsum("j,ekji...->eki...", w, x5)                    # (k2 = k, k1 = i)
        else:
            y = np.einsum("k,ekji...->eji...", w, x5)                    # (k2 = j, k1 = i)
        return y.reshape((x.shape[0], n1 * n1) + x.shape[2:])

    def traces(self, q):
        return np.stack([self.face_interp(q, f) for f in range(6)], axis=1)   # [Ne, 6, nf, Nv]

    def neighbour_face_values(self, x):
        """The neighbour's values on each shared face, in this face's point order (zero on
        boundary faces); x [Ne, 6, nf, ...]."""
        m = self.mesh
        out = np.zeros_like(x)
        for f in range(6):
            nb = m.face_nbr[:, f]
            inner = nb >= 0
            idx = np.where(inner, nb, 0)
            vals = x[idx, m.face_nbr_face[:, f]]                           # [Ne, nf, ...]
            perm = self._omaps[m.face_orient[:, f]]                        # [Ne, nf]
            vals = np.take_along_axis(vals, perm.reshape(perm.shape + (1,) * (vals.ndim - 2)), axis=1)
            out[:, f] = np.where(inner.reshape((-1,) + (1,) * (vals.ndim - 1)), vals, 0.0)
        return out

    def outside_states(self, own, nbr_tr):
        m = self.mesh
        out = self.neighbour_face_values(nbr_tr).astype(np.result_type(own, nbr_tr))
        for f in range(6):
            nb = m.face_nbr[:, f]
            wall = nb == BC_SLIP_WALL
            if np.any(wall):
                nvec = self.geo.fvec[:, f]
                nunit = nvec / np.sqrt(np.sum(nvec * nvec, axis=-1))[..., None]
                u = own[:, f, :, 1:4]
                un = np.sum(u * nunit, axis=-1)
                ghost = own[:, f].copy()
                ghost[..., 1:4] = u - 2.0 * un[..., None] * nunit
                out[:, f] = np.where(wall[:, None, None], ghost, out[:, f])
            far = nb == BC_FAR_FIELD
            if np.any(far):
                out[:, f] = np.where(far[:, None, None], self.q_inf, out[:, f])
        return out

    # ---- residual ----------------------------------------------------------------
    def residual(self, q, q_nbr=None):
        """R(q) at the solution points, [Ne, Np, Nv] (q_nbr: the state the neighbours' traces
        are taken from, default q)."""
        o, g, ne, n1, nv = self.ops, self.geo, self.ne, self.n1, self.nv
        own = self.traces(q)
        nbr_tr = own if q_nbr is None else self.traces(q_nbr)
        out = self.outside_states(own, nbr_tr)
        ft = [G.normal_flux(q, g.Ja[:, d], self.gas) for d in range(3)]          # [Ne, Np, Nv]
        div = np.zeros((ne, n1, n1, n1, nv), dtype=np.result_type(q, own))
        for d in range(3):
            F5 = ft[d].reshape(ne, n1, n1, n1, nv)                             # [e, k, j, i, v]
            if d == 0:
                div = div + np.einsum("im,ekjmv->ekjiv", o.D, F5)
            elif d == 1:
                div = div + np.einsum("jm,ekmiv->ekjiv", o.D, F5)
            else:
                div = div + np.einsum("km,emjiv->ekjiv", o.D, F5)
            for side in (0, 1):
                f = 2 * d + side
                fv = g.fvec[:, f]
                if side == 0:
                    fh = G.common_flux(out[:, f], own[:, f], fv, self.gas)
                else:
                    fh = G.common_flux(own[:, f], out[:, f], fv, self.gas)
                jump = (fh - self.face_interp(ft[d], f)).reshape(ne, n1, n1, nv)   # [e, k2, k1, v]
                gp = o.gL if side == 0 else o.gR
                if d == 0:      # (k2, k1) = (k, j); line along i
                    div = div + gp[None, None, None, :, None] * jump[:, :, :, None, :]
                elif d == 1:    # (k2, k1) = (k, i); line along j
                    div = div + gp[None, None, :, None, None] * jump[:, :, None, :, :]
                else:           # (k2, k1) = (j, i); line along k
                    div = div + gp[None, :, None, None, None] * jump[:, None, :, :, :]
        return -div.reshape(ne, self.npts, nv) / g.jac[..., None]

    def stage_residual(self, q, c_mass=0.0, src=None, S=None, q_nbr=None):
        """F(q) - S with F = R(q) - c_mass q_c(q) + src (eq. (26))."""
        F = self.residual(q, q_nbr)
        if c_mass != 0.0:
            F = F - c_mass * G.conservative(q, self.gas)
        if src is not None:
            F = F + src
        if S is not None:
            F = F - S
        return F
