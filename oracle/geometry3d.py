"""Element mappings and metric terms for hexahedral FR/CPR levels (Sec. 2.3, three dimensions).

The mapping x(xi, eta, zeta) is the Lagrange interpolant of the element's geometry nodes
(trilinear for order 1, 27-node triquadratic for order 2). The transformed flux in reference
direction i is f . (J grad xi^i); in three dimensions these metric vectors (J grad xi = x_eta x
x_zeta and cyclic) are products of degree higher than P on curved elements, and their plain
interpolants do not satisfy the discrete metric identities, so a uniform flow would not stay
uniform. Reading (the paper states no metric treatment): the metric terms are taken in the
conservative curl form of Kopriva (2006),

  (J grad xi^i)_n = -[curl_xi (I_Q (X_l grad_xi X_m))]_i,   (n, m, l) cyclic,

with I_Q the tensor-product interpolant at the Q+1 Gauss-Lobatto points (Q = max(P, 1)). The curl
of that interpolant is a polynomial of degree <= Q in each reference direction, so for P >= 1 its
values at the (P+1)^3 Gauss points represent it exactly (the discrete divergence of the metric
terms vanishes) and its value on a face depends only on the face's geometry (the two elements of
a face get the same face vector). The face vectors at the flux points are that same polynomial
evaluated on the face. The Jacobian |J| at the solution points is that of the exact mapping.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from .basis import Ops1D, lagrange_deriv, lagrange_eval


def gauss_lobatto_points(Q: int) -> np.ndarray:
    """The Q+1 Gauss-Lobatto points on [-1, 1]: the ends and the roots of L_Q'."""
    c = np.zeros(Q + 1)
    c[Q] = 1.0
    inner = npleg.legroots(npleg.legder(c)) if Q >= 2 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def map_and_derivs(nodes: np.ndarray, g: int, pts: np.ndarray):
    """x and dx/dxi^k at reference points pts [m, 3] of every element: [Ne, m, 3] and
    [Ne, m, 3 (x component), 3 (k)]. Node a + (g+1) b + (g+1)^2 c sits at the g-uniform grid."""
    gn = np.linspace(-1.0, 1.0, g + 1)
    L = [lagrange_eval(gn, pts[:, d]) for d in range(3)]        # [m, g+1]
    dL = [lagrange_deriv(gn, pts[:, d]) for d in range(3)]
    sh = np.einsum("ma,mb,mc->mcba", L[0], L[1], L[2]).reshape(len(pts), -1)
    dsh = [np.einsum("ma,mb,mc->mcba", dL[0], L[1], L[2]).reshape(len(pts), -1),
           np.einsum("ma,mb,mc->mcba", L[0], dL[1], L[2]).reshape(len(pts), -1),
           np.einsum("ma,mb,mc->mcba", L[0], L[1], dL[2]).reshape(len(pts), -1)]
    x = np.einsum("mk,ekd->emd", sh, nodes)
    dx = np.stack([np.einsum("mk,ekd->emd", s, nodes) for s in dsh], axis=-1)
    return x, dx


def tensor_points(x1: np.ndarray) -> np.ndarray:
    """Points (x1[i], x1[j], x1[k]) in the order p = i + n j + n^2 k."""
    n = len(x1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([x1[i.ravel()], x1[j.ravel()], x1[k.ravel()]], axis=-1)


def face_coords(f: int, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """Reference points of face f for tangential coordinates (t1, t2) (arrays of equal length)."""
    s = -1.0 if f % 2 == 0 else 1.0
    c = np.full(len(t1), s)
    if f < 2:
        return np.stack([c, t1, t2], axis=-1)
    if f < 4:
        return np.stack([t1, c, t2], axis=-1)
    return np.stack([t1, t2, c], axis=-1)


class HexGeometry:
    """Metrics of one P-level on a hexahedral mesh.

    Attributes (Ne elements, Np = (P+1)^3 solution points, p = i + (P+1) j + (P+1)^2 k):
      xyz   [Ne, Np, 3] physical solution-point coordinates
      Ja    [Ne, 3, Np, 3] metric vector J grad xi^d of reference direction d at solution points
      jac   [Ne, Np] |J| of the exact mapping
      fvec  [Ne, 6, (P+1)^2, 3] +xi^d vector (d = f // 2) at the face points k1 + (P+1) k2
    """

    def __init__(self, mesh, P: int):
        assert mesh.dim == 3
        self.P = P
        ops = Ops1D(P)
        n1 = P + 1
        g = mesh.geom_order
        ne = mesh.n_elements
        sp = tensor_points(ops.x)
        self.xyz, dx = map_and_derivs(mesh.nodes, g, sp)
        self.jac = np.linalg.det(dx)
        # curl-form metrics at the Gauss-Lobatto grid
        Q = max(P, 1)
        y = gauss_lobatto_points(Q)
        nq = Q + 1
        xg, dxg = map_and_derivs(mesh.nodes, g, tensor_points(y))
        Dg = lagrange_deriv(y, y)

        def dref(u, d):
            """Derivative along reference direction d of grid values u [Ne, nq^3, ...]."""
            u5 = u.reshape((ne, nq, nq, nq) + u.shape[2:])          # [e, k, j, i, ...]
            axis = {0: 3, 1: 2, 2: 1}[d]
            out = np.moveaxis(np.tensordot(Dg, np.moveaxis(u5, axis, 0), axes=(1, 0)), 0, axis)
            return out.reshape(u.shape)

        Ja_gl = np.zeros((ne, 3, nq ** 3, 3))                        # [e, i, grid, n]
        for n in range(3):
            m, l = (n + 1) % 3, (n + 2) % 3
            V = xg[..., l][..., None] * dxg[:, :, m, :]                # V_k = X_l dX_m/dxi^k
            curl = [dref(V[..., 2], 1) - dref(V[..., 1], 2),
                    dref(V[..., 0], 2) - dref(V[..., 2], 0),
                    dref(V[..., 1], 0) - dref(V[..., 0], 1)]
            for i in range(3):
                Ja_gl[:, i, :, n] = -curl[i]
        # the polynomial at the Gauss points and at the face points
        Lv = lagrange_eval(y, ops.x)                                  # [n1, nq]
        J5 = Ja_gl.reshape(ne, 3, nq, nq, nq, 3)                     # [e, i, k, j, a, n]
        Jsp = np.einsum("ia,jb,kc,edcban->edkjin", Lv, Lv, Lv, J5)
        self.Ja = Jsp.reshape(ne, 3, n1 ** 3, 3)
        self.fvec = np.zeros((ne, 6, n1 * n1, 3))
        for f in range(6):
            d = f // 2
            end = 0 if f % 2 == 0 else Q
            Jd = J5[:, d]                                             # [e, k, j, a, n]
            if d == 0:
                face = Jd[:, :, :, end]                               # [e, k(t2), j(t1), n]
            elif d == 1:
                face = Jd[:, :, end, :]                               # [e, k(t2), a(t1), n]
            else:
                face = Jd[:, end]                                     # [e, j(t2), a(t1), n]
            vals = np.einsum("xa,yb,ebad->eyxd", Lv, Lv, face)        # [e, k2, k1, n]
            self.fvec[:, f] = vals.reshape(ne, n1 * n1, 3)


def element_dx3(mesh, nq: int = 5) -> np.ndarray:
    """Delta x of eqs. (32)-(33) on hexahedra: twice the minimum distance from each element's
    volume centroid (nq^3 Gauss rule of the exact mapping) to its faces. Reading: the distance to
    a face is the distance to the plane through the face's centre node with the normal of the
    cross product of the face's corner diagonals."""
    from .basis import gauss_points
    g = mesh.geom_order
    xq, wq = gauss_points(nq - 1)
    pts = tensor_points(xq)
    w = np.einsum("k,j,i->kji", wq, wq, wq).ravel()
    x, dx = map_and_derivs(mesh.nodes, g, pts)
    jac = np.linalg.det(dx)
    vol = jac @ w
    cen = np.einsum("em,m,emd->ed", jac, w, x) / vol[:, None]
    n1 = g + 1

    def idx(a, b, c):
        return a + n1 * b + n1 * n1 * c

    h = g // 2 if g % 2 == 0 else None
    dmin = np.full(mesh.n_elements, np.inf)
    for f in range(6):
        end = 0 if f % 2 == 0 else g
        if f < 2:
            corners = [idx(end, 0, 0), idx(end, g, 0), idx(end, g, g), idx(end, 0, g)]
        elif f < 4:
            corners = [idx(0, end, 0), idx(g, end, 0), idx(g, end, g), idx(0, end, g)]
        else:
            corners = [idx(0, 0, end), idx(g, 0, end), idx(g, g, end), idx(0, g, end)]
        c = mesh.nodes[:, corners]
        nrm = np.cross(c[:, 2] - c[:, 0], c[:, 3] - c[:, 1])
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        if h is not None:
            mid = {0: idx(0, h, h), 1: idx(g, h, h), 2: idx(h, 0, h), 3: idx(h, g, h),
                   4: idx(h, h, 0), 5: idx(h, h, g)}[f]
            p0 = mesh.nodes[:, mid]
        else:
            p0 = c.mean(axis=1)
        d = np.abs(np.sum((cen - p0) * nrm, axis=1))
        dmin = np.minimum(dmin, d)
    return 2.0 * dmin
