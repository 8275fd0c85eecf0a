"""Ideal-gas relations, the Weiss-Smith preconditioner and the common inviscid flux.

All functions are vectorised over leading axes; the last axis holds the primitive
working variables q_p = (p, u_1..u_d, T) (Sec. 2.2). Every function accepts complex
input and is complex-analytic in it (|x| and min/max are taken on the real part), so
the Jacobian module can differentiate through it by the complex step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Gas:
    gamma: float = 1.4
    rgas: float = 1.0
    prandtl: float = 0.72
    mu: float = 0.0
    # reference-velocity model of eq. (11): mode "local" uses eps = min(1, Ma) (the
    # cut-off switched off, as for the vortex in Sec. 4.1); mode "cutoff" uses
    # eps = min(1, max(kappa*Ma_inf, Ma)).
    eps_mode: str = "local"
    ma_inf: float = 0.0
    kappa: float = 1.0
    # penalty of the BR2 common gradient (oracle.viscous)
    br2_penalty: float = 4.0

    @property
    def cp(self) -> float:
        return self.gamma * self.rgas / (self.gamma - 1.0)


def rabs(x):
    """|x| continued analytically from the real axis."""
    return np.where(np.real(x) < 0, -x, x)


def rmin(a, b):
    return np.where(np.real(a) <= np.real(b), a, b)


def rmax(a, b):
    return np.where(np.real(a) >= np.real(b), a, b)


def _split(q):
    return q[..., 0], q[..., 1:-1], q[..., -1]


def density(q, gas: Gas):
    """Ideal-gas law p = rho R T (Sec. 2.1)."""
    p, _, T = _split(q)
    return p / (gas.rgas * T)


def specific_energy(q, gas: Gas):
    """E = (p/rho)/(gamma-1) + u.u/2 (Sec. 2.1)."""
    p, u, _ = _split(q)
    rho = density(q, gas)
    return (p / rho) / (gas.gamma - 1.0) + 0.5 * np.sum(u * u, axis=-1)


def total_enthalpy(q, gas: Gas):
    """H = E + p/rho (Sec. 2.1)."""
    p, _, _ = _split(q)
    return specific_energy(q, gas) + p / density(q, gas)


def conservative(q, gas: Gas):
    """q_c = (rho, rho u_i, rho E)."""
    rho = density(q, gas)
    _, u, _ = _split(q)
    return np.concatenate([rho[..., None], rho[..., None] * u,
                           (rho * specific_energy(q, gas))[..., None]], axis=-1)


def primitive(qc, gas: Gas):
    """Inverse of ``conservative``: (rho, rho u_i, rho E) -> (p, u_i, T) with p from the total
    energy, p = (gamma - 1)(rho E - rho |u|^2 / 2), and T = p / (rho R) (ideal gas, Sec. 2.1)."""
    rho = qc[..., 0]
    u = qc[..., 1:-1] / rho[..., None]
    p = (gas.gamma - 1.0) * (qc[..., -1] - 0.5 * rho * np.sum(u * u, axis=-1))
    return np.concatenate([p[..., None], u, (p / (rho * gas.rgas))[..., None]], axis=-1)


def sound_speed(q, gas: Gas):
    _, _, T = _split(q)
    return np.sqrt(gas.gamma * gas.rgas * T)


def mass_matrix(q, gas: Gas):
    """M = d q_c / d q_p (Sec. 2.2, eq. (8)), differentiated term by term from q_c above."""
    p, u, T = _split(q)
    d = u.shape[-1]
    nv = d + 2
    rho = density(q, gas)
    rho_p = 1.0 / (gas.rgas * T)
    rho_T = -p / (gas.rgas * T * T)
    ke = 0.5 * np.sum(u * u, axis=-1)
    M = np.zeros(q.shape[:-1] + (nv, nv), dtype=q.dtype)
    M[..., 0, 0] = rho_p
    M[..., 0, -1] = rho_T
    for i in range(d):
        M[..., 1 + i, 0] = rho_p * u[..., i]
        M[..., 1 + i, 1 + i] = rho
        M[..., 1 + i, -1] = rho_T * u[..., i]
        M[..., -1, 1 + i] = rho * u[..., i]
    M[..., -1, 0] = 1.0 / (gas.gamma - 1.0) + rho_p * ke
    M[..., -1, -1] = rho_T * ke
    return M


def epsilon(q, gas: Gas):
    """Reference-velocity factor eps of eq. (11) (U_r = eps c)."""
    _, u, _ = _split(q)
    ma = np.sqrt(np.sum(u * u, axis=-1)) / sound_speed(q, gas)
    if gas.eps_mode == "local":
        return rmin(np.ones_like(ma), ma)
    if gas.eps_mode == "cutoff":
        return rmin(np.ones_like(ma), rmax(gas.kappa * gas.ma_inf * np.ones_like(ma), ma))
    raise ValueError(gas.eps_mode)


def preconditioner(q, gas: Gas, eps=None):
    """Weiss-Smith preconditioning matrix Gamma, eq. (9), with Theta of eq. (10)."""
    p, u, T = _split(q)
    d = u.shape[-1]
    nv = d + 2
    if eps is None:
        eps = epsilon(q, gas)
    rho = density(q, gas)
    rho_T = -p / (gas.rgas * T * T)
    H = total_enthalpy(q, gas)
    ur = eps * sound_speed(q, gas)
    theta = 1.0 / (ur * ur) - rho_T / (rho * gas.cp)
    G = np.zeros(q.shape[:-1] + (nv, nv), dtype=q.dtype)
    G[..., 0, 0] = theta
    G[..., 0, -1] = rho_T
    for i in range(d):
        G[..., 1 + i, 0] = theta * u[..., i]
        G[..., 1 + i, 1 + i] = rho
        G[..., 1 + i, -1] = rho_T * u[..., i]
        G[..., -1, 1 + i] = rho * u[..., i]
    G[..., -1, 0] = theta * H - 1.0
    G[..., -1, -1] = rho_T * H + rho * gas.cp
    return G


def normal_flux(q, nvec, gas: Gas):
    """Inviscid flux f.n for a (not necessarily unit) vector n (Sec. 2.1, eqs. (1)-(3))."""
    p, u, _ = _split(q)
    rho = density(q, gas)
    un = np.sum(u * nvec, axis=-1)
    H = total_enthalpy(q, gas)
    mom = rho[..., None] * u * un[..., None] + p[..., None] * nvec
    return np.concatenate([(rho * un)[..., None], mom, (rho * H * un)[..., None]], axis=-1)


def flux_jacobian(q, nvec, gas: Gas):
    """A_n = d(f.n)/d q_p, differentiated term by term from ``normal_flux``."""
    p, u, T = _split(q)
    d = u.shape[-1]
    nv = d + 2
    rho = density(q, gas)
    rho_p = 1.0 / (gas.rgas * T)
    rho_T = -p / (gas.rgas * T * T)
    un = np.sum(u * nvec, axis=-1)
    H = total_enthalpy(q, gas)
    A = np.zeros(q.shape[:-1] + (nv, nv), dtype=np.result_type(q, nvec))
    A[..., 0, 0] = rho_p * un
    A[..., 0, -1] = rho_T * un
    A[..., -1, 0] = rho_p * H * un
    A[..., -1, -1] = (rho_T * H + rho * gas.cp) * un
    for k in range(d):
        A[..., 0, 1 + k] = rho * nvec[..., k]
        A[..., -1, 1 + k] = rho * (u[..., k] * un + H * nvec[..., k])
    for i in range(d):
        A[..., 1 + i, 0] = rho_p * u[..., i] * un + nvec[..., i]
        A[..., 1 + i, -1] = rho_T * u[..., i] * un
        for k in range(d):
            A[..., 1 + i, 1 + k] = rho * (u[..., i] * nvec[..., k] + (un if i == k else 0.0))
    return A


def preconditioned_eigenvalues(q, nunit, gas: Gas, eps=None):
    """The three distinct eigenvalues of Gamma^{-1} A_n for a unit normal, eq. (13):
    u_n (multiplicity d), u_n(1-alpha) + c', u_n(1-alpha) - c'."""
    p, u, T = _split(q)
    if eps is None:
        eps = epsilon(q, gas)
    rho = density(q, gas)
    rho_p = 1.0 / (gas.rgas * T)
    rho_T = -p / (gas.rgas * T * T)
    beta = rho_p + rho_T / (rho * gas.cp)
    ur = eps * sound_speed(q, gas)
    alpha = 0.5 * (1.0 - beta * ur * ur)
    un = np.sum(u * nunit, axis=-1)
    cprime = np.sqrt(alpha * alpha * un * un + ur * ur)
    return un, un * (1.0 - alpha) + cprime, un * (1.0 - alpha) - cprime


def common_flux(qm, qp, svec, gas: Gas):
    """Common inviscid normal flux of eq. (21), scaled by |S|.

    ``qm`` is the '-' (left) state, ``qp`` the '+' (right) state and ``svec`` a vector
    pointing from left to right whose length is the face area element; the return
    value is |S| f_com(q-, q+; S/|S|).

    Readings: the averaged state of eq. (21) is the arithmetic mean of the primitive
    variables, and eps (hence U_r) is evaluated from that mean; no entropy fix.
    |Gamma^{-1} A_n| = R |Lambda| R^{-1} is formed from its spectral projectors
    (Sylvester's formula over the three distinct eigenvalues), the textbook
    definition of a function of a diagonalisable matrix.
    """
    smag = np.sqrt(np.sum(svec * svec, axis=-1))
    nunit = svec / smag[..., None]
    qa = 0.5 * (qm + qp)
    eps = epsilon(qa, gas)
    G = preconditioner(qa, gas, eps)
    A = flux_jacobian(qa, nunit, gas)
    X = np.linalg.solve(G, A)
    lams = preconditioned_eigenvalues(qa, nunit, gas, eps)
    eye = np.eye(qm.shape[-1])
    absX = np.zeros_like(X)
    for k in range(3):
        proj = np.broadcast_to(eye, X.shape).astype(X.dtype)
        for j in range(3):
            if j != k:
                proj = ((X - lams[j][..., None, None] * eye) @ proj) / (lams[k] - lams[j])[..., None, None]
        absX = absX + rabs(lams[k])[..., None, None] * proj
    dq = (qp - qm)[..., None]
    diss = (G @ (absX @ dq))[..., 0]
    fc = 0.5 * (normal_flux(qm, nunit, gas) + normal_flux(qp, nunit, gas)) - 0.5 * diss
    return smag[..., None] * fc
