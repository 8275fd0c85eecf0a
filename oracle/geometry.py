"""Element mappings and metric terms for quadrilateral FR/CPR levels (Sec. 2.3).

The mapping x(xi, eta) is the Lagrange interpolant of the element's geometry
nodes (bilinear for order 1, 9-node biquadratic for order 2). Metrics are taken
from that exact mapping at the solution and flux points of every P-level
(coarse levels re-discretise the same geometry).

For a quad the contravariant fluxes are F~ = |J|(xi_x f + xi_y g) = y_eta f - x_eta g
and G~ = |J|(eta_x f + eta_y g) = -y_xi f + x_xi g, so the transformed flux in the
+xi direction is f.S with S = (y_eta, -x_eta), and in the +eta direction f.T with
T = (-y_xi, x_xi).
"""
from __future__ import annotations

import numpy as np

from .basis import Ops1D, lagrange_deriv, lagrange_eval


def _map_derivs(nodes: np.ndarray, g: int, xi: np.ndarray, eta: np.ndarray):
    """x, x_xi, x_eta at reference points (xi[m], eta[m]) of every element.

    nodes: [Ne, (g+1)^2, 2]; returns arrays [Ne, m, 2].
    """
    gn = np.linspace(-1.0, 1.0, g + 1)
    Nx, Ny = lagrange_eval(gn, xi), lagrange_eval(gn, eta)      # [m, g+1]
    dNx, dNy = lagrange_deriv(gn, xi), lagrange_deriv(gn, eta)
    # shape function of node a + (g+1) b is N_a(xi) N_b(eta)
    sh = np.einsum("ma,mb->mba", Nx, Ny).reshape(xi.size, -1)
    sh_xi = np.einsum("ma,mb->mba", dNx, Ny).reshape(xi.size, -1)
    sh_eta = np.einsum("ma,mb->mba", Nx, dNy).reshape(xi.size, -1)
    x = np.einsum("mk,ekd->emd", sh, nodes)
    x_xi = np.einsum("mk,ekd->emd", sh_xi, nodes)
    x_eta = np.einsum("mk,ekd->emd", sh_eta, nodes)
    return x, x_xi, x_eta


class QuadGeometry:
    """Metrics of one P-level on a quad mesh.

    Attributes (Ne elements, Np = (P+1)^2 solution points, p = i + (P+1) j):
      xy     [Ne, Np, 2] physical solution-point coordinates
      S_sp   [Ne, Np, 2] xi-direction vector (y_eta, -x_eta) at solution points
      T_sp   [Ne, Np, 2] eta-direction vector (-y_xi, x_xi) at solution points
      jac    [Ne, Np]    |J|
      fvec   [Ne, 4, P+1, 2] +xi (faces 0, 1) or +eta (faces 2, 3) vector at flux points
    """

    def __init__(self, mesh, P: int):
        self.P = P
        ops = Ops1D(P)
        n1 = P + 1
        g = mesh.geom_order
        x1 = ops.x
        ii, jj = np.meshgrid(np.arange(n1), np.arange(n1), indexing="xy")  # p = i + n1 j
        xi = x1[ii.ravel()]
        eta = x1[jj.ravel()]
        xy, dxi, deta = _map_derivs(mesh.nodes, g, xi, eta)
        self.xy = xy
        x_xi, y_xi = dxi[..., 0], dxi[..., 1]
        x_eta, y_eta = deta[..., 0], deta[..., 1]
        self.S_sp = np.stack([y_eta, -x_eta], axis=-1)
        self.T_sp = np.stack([-y_xi, x_xi], axis=-1)
        self.jac = x_xi * y_eta - x_eta * y_xi
        ne = mesh.n_elements
        self.fvec = np.zeros((ne, 4, n1, 2))
        one = np.ones(n1)
        for f, (fx, fe) in enumerate([(-one, x1), (one, x1), (x1, -one), (x1, one)]):
            _, dxi_f, deta_f = _map_derivs(mesh.nodes, g, fx, fe)
            if f < 2:
                self.fvec[:, f] = np.stack([deta_f[..., 1], -deta_f[..., 0]], axis=-1)
            else:
                self.fvec[:, f] = np.stack([-dxi_f[..., 1], dxi_f[..., 0]], axis=-1)


def element_dx(mesh, nq: int = 6) -> np.ndarray:
    """Delta x of eqs. (32)-(33): twice the minimum distance from each element's barycentre to its
    faces. Reading: the barycentre is the area centroid of the exact mapping (nq x nq Gauss rule);
    the distance to a face is the distance to the segment joining the face's two corner nodes."""
    from .basis import gauss_points
    g = mesh.geom_order
    xq, wq = gauss_points(nq - 1)
    ii, jj = np.meshgrid(np.arange(nq), np.arange(nq), indexing="xy")
    xi, eta = xq[ii.ravel()], xq[jj.ravel()]
    w = (wq[:, None] * wq[None, :]).T.ravel()          # weight of point i + nq j is w_i w_j
    x, dxi, deta = _map_derivs(mesh.nodes, g, xi, eta)
    jac = dxi[..., 0] * deta[..., 1] - deta[..., 0] * dxi[..., 1]
    area = jac @ w
    cen = np.einsum("em,m,emd->ed", jac, w, x) / area[:, None]
    n1 = g + 1
    corner = {0: (0, n1 * g), 1: (g, g + n1 * g), 2: (0, g), 3: (n1 * g, g + n1 * g)}
    dmin = np.full(mesh.n_elements, np.inf)
    for f, (a, b) in corner.items():
        pa, pb = mesh.nodes[:, a], mesh.nodes[:, b]
        ab = pb - pa
        t = np.clip(np.sum((cen - pa) * ab, axis=1) / np.sum(ab * ab, axis=1), 0.0, 1.0)
        d = np.linalg.norm(cen - (pa + t[:, None] * ab), axis=1)
        dmin = np.minimum(dmin, d)
    return 2.0 * dmin
