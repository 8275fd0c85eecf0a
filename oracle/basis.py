"""1-D reference-element operators for tensor-product FR/CPR (Sec. 2.3).

Readings: solution points are the P+1 Gauss-Legendre points per direction and the
flux points on a face are the same 1-D points (the paper does not name its point
set). The 1-D correction function is Huynh's g_DG, the right Radau polynomial,
for which FR recovers nodal DG (the paper only says the correction field is a
tensor product of 1-D correction polynomials).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_points(P: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre points and weights on [-1, 1], P+1 of them."""
    x, w = npleg.leggauss(P + 1)
    return x, w


def lagrange_eval(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Matrix L[m, k] = l_k(x_m) of the Lagrange basis on ``nodes``."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    out = np.ones((x.size, nodes.size))
    for k in range(nodes.size):
        for m in range(nodes.size):
            if m != k:
                out[:, k] *= (x - nodes[m]) / (nodes[k] - nodes[m])
    return out


def lagrange_deriv(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Matrix D[m, k] = l_k'(x_m), by the product rule on l_k = prod (x - x_s)/(x_k - x_s)."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = nodes.size
    out = np.zeros((x.size, n))
    for k in range(n):
        for s in range(n):
            if s == k:
                continue
            term = np.full(x.size, 1.0 / (nodes[k] - nodes[s]))
            for m in range(n):
                if m != k and m != s:
                    term = term * (x - nodes[m]) / (nodes[k] - nodes[m])
            out[:, k] += term
    return out


def radau_right_deriv(P: int, x: np.ndarray) -> np.ndarray:
    """g_R'(x) for g_R = (L_{P+1} + L_P)/2: g_R(1) = 1, g_R(-1) = 0, g_R orthogonal to P_{P-1}."""
    c = np.zeros(P + 2)
    c[P + 1] = 0.5
    c[P] = 0.5
    return npleg.legval(np.asarray(x, float), npleg.legder(c))


def radau_left_deriv(P: int, x: np.ndarray) -> np.ndarray:
    """g_L'(x) for the mirror image g_L(x) = g_R(-x)."""
    return -radau_right_deriv(P, -np.asarray(x, float))


class Ops1D:
    """The 1-D operators of one polynomial degree P on Gauss points."""

    def __init__(self, P: int):
        self.P = P
        self.n1 = P + 1
        self.x, self.w = gauss_points(P)
        self.D = lagrange_deriv(self.x, self.x)                # D[i, k] = l_k'(x_i)
        self.lm = lagrange_eval(self.x, np.array([-1.0]))[0]   # l_k(-1)
        self.lp = lagrange_eval(self.x, np.array([1.0]))[0]    # l_k(+1)
        self.gL = radau_left_deriv(P, self.x)                  # g_L'(x_i)
        self.gR = radau_right_deriv(P, self.x)                 # g_R'(x_i)


def projection_1d(Pf: int, Pc: int) -> np.ndarray:
    """Restriction 1-D matrix: L2 projection of the degree-Pf polynomial through the fine
    Gauss values onto degree Pc, sampled at the coarse Gauss points (Sec. 3, eqs. (39), (40)).

    Legendre coefficients a_k = (2k+1)/2 * sum_i w_i L_k(x_i) u_i are exact for k <= Pf with
    Pf+1 Gauss points; the modes k <= Pc are kept and evaluated at the coarse points.
    Reading: the projection is taken in the reference element (not |J|-weighted).
    """
    xf, wf = gauss_points(Pf)
    xc, _ = gauss_points(Pc)
    Vf = npleg.legvander(xf, Pc)           # [nf, Pc+1]
    Vc = npleg.legvander(xc, Pc)           # [nc, Pc+1]
    scale = (2.0 * np.arange(Pc + 1) + 1.0) / 2.0
    return Vc @ (scale[:, None] * (Vf * wf[:, None]).T)


def interpolation_1d(Pc: int, Pf: int) -> np.ndarray:
    """Prolongation 1-D matrix: the coarse polynomial evaluated at the fine points (eqs. (44), (45))."""
    xc, _ = gauss_points(Pc)
    xf, _ = gauss_points(Pf)
    return lagrange_eval(xc, xf)
