"""Pins of the oracle's BR2 viscous terms (Sec. 2.1 fluxes, Sec. 2.3 eqs. (22)-(23))."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle import solver as OS
from oracle.basis import gauss_points
from oracle.fr import FRLevel
from oracle.jacobian import element_dFdq
from oracle.viscous import viscous_flux


def vgas(mu=0.3, ma=0.1, penalty=4.0):
    return G.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=ma, kappa=1.0, mu=mu, br2_penalty=penalty)


def weights(P, lev):
    _, w = gauss_points(P)
    return lev.geo.jac * np.outer(w, w).ravel()[None, :]


def test_viscous_flux_closed_forms():
    """Pure extension, pure shear and pure conduction against the stress and heat-flux
    definitions of Sec. 2.1 (tau = 2 mu (S - div u / 3 I), K = -mu C_p / Pr grad T)."""
    gas = vgas(mu=0.7)
    q = np.array([10.0, 2.0, -3.0, 5.0])
    k = 0.7 * gas.cp / gas.prandtl
    g = np.zeros((4, 2))
    g[1, 0] = 1.0                                    # u_x = 1
    fx, fy = viscous_flux(q, g, gas)
    assert np.allclose(fx, [0, 4 / 3 * 0.7, 0, 2.0 * 4 / 3 * 0.7], rtol=1e-15)
    assert np.allclose(fy, [0, 0, -2 / 3 * 0.7, -3.0 * -2 / 3 * 0.7], rtol=1e-15)
    g = np.zeros((4, 2))
    g[1, 1] = 1.0                                    # u_y = 1: tau_xy = mu
    fx, fy = viscous_flux(q, g, gas)
    assert np.allclose(fx, [0, 0, 0.7, -3.0 * 0.7], rtol=1e-15)
    assert np.allclose(fy, [0, 0.7, 0, 2.0 * 0.7], rtol=1e-15)
    g = np.zeros((4, 2))
    g[3, 1] = 1.0                                    # T_y = 1: energy flux k in y
    fx, fy = viscous_flux(q, g, gas)
    assert np.allclose(fx, 0.0) and np.allclose(fy, [0, 0, 0, k], rtol=1e-15)


def _linear_operator(lev, lev0, base, var_in, var_out):
    """Matrix of the viscous residual's component var_out as a function of var_in (all other
    unknowns fixed at base), by unit perturbations (the map is affine)."""
    ne, npts = lev.ne, lev.npts
    n = ne * npts
    r0 = (lev.residual(base) - lev0.residual(base))[..., var_out].reshape(n)
    A = np.zeros((n, n))
    for c in range(n):
        q = base.copy()
        q.reshape(n, 4)[c, var_in] += 1.0
        A[:, c] = (lev.residual(q) - lev0.residual(q))[..., var_out].reshape(n) - r0
    return A


@pytest.mark.parametrize("P,jitter", [(2, 0.0), (2, 0.15), (3, 0.15)])
def test_heat_conduction_operator_is_symmetric_negative(P, jitter):
    """At rest, the BR2 energy residual is the discrete div(k grad T): in the quadrature inner
    product (weights w |J|) it must be symmetric and negative semi-definite with the constants
    as its null space, on distorted periodic meshes. A lifting with the wrong sign or scale, or
    an unsymmetric common gradient, breaks this."""
    mesh = W.periodic_rect_mesh(4, 3, 4.0, 3.0, jitter=jitter, seed=2)
    lev, lev0 = FRLevel(mesh, P, vgas()), FRLevel(mesh, P, vgas(mu=0.0))
    base = np.zeros((lev.ne, lev.npts, 4))
    base[..., 0], base[..., 3] = 100.0, 80.0
    A = _linear_operator(lev, lev0, base, 3, 3)
    B = weights(P, lev).reshape(-1)[:, None] * A
    scale = np.abs(B).max()
    assert np.abs(B - B.T).max() <= 1e-12 * scale
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev.max() <= 1e-12 * scale
    assert np.sum(ev > -1e-9 * scale) == 1              # one zero eigenvalue: the constants
    assert np.abs(A.sum(axis=1)).max() <= 1e-10 * np.abs(A).max()


def curved_periodic_mesh(n=3, L=3.0, amp=0.08):
    """Periodic box of biquadratic elements whose nodes are moved by a smooth periodic field."""
    m = W.periodic_rect_mesh(n, n, L, L, ox=0.0, oy=0.0)
    h = L / n
    nodes = np.zeros((m.n_elements, 9, 2))
    for e in range(m.n_elements):
        i, j = e % n, e // n
        for b in range(3):
            for a in range(3):
                x, y = (i + a / 2) * h, (j + b / 2) * h
                nodes[e, a + 3 * b] = (x + amp * np.sin(2 * np.pi * y / L) * np.sin(2 * np.pi * x / L),
                                       y + amp * np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L))
    return W.Mesh(2, 2, nodes, m.face_nbr, m.face_nbr_face, m.face_orient)


@pytest.mark.parametrize("case", ["curved_periodic", "far_field_box"])
def test_heat_operator_symmetric_on_curved_elements_and_far_field(case):
    """The same symmetry on biquadratic (curved) elements, and with far-field boundaries, where
    q_com is the free stream itself (the mean with the ghost would break it); there the
    boundary makes the operator negative definite."""
    if case == "curved_periodic":
        mesh = curved_periodic_mesh()
    else:
        mesh = W.channel_mesh(4, 3, 4.0, 3.0, jitter=0.1, seed=2, wall=W.BC_FAR_FIELD)
    q_inf = np.array([100.0, 0.0, 0.0, 80.0])
    lev, lev0 = FRLevel(mesh, 3, vgas(), q_inf=q_inf), FRLevel(mesh, 3, vgas(mu=0.0), q_inf=q_inf)
    assert np.all(lev.geo.jac > 0)
    base = np.zeros((lev.ne, lev.npts, 4))
    base[..., 0], base[..., 3] = 100.0, 80.0
    A = _linear_operator(lev, lev0, base, 3, 3)
    B = weights(3, lev).reshape(-1)[:, None] * A
    scale = np.abs(B).max()
    assert np.abs(B - B.T).max() <= 1e-12 * scale
    top = np.linalg.eigvalsh(0.5 * (B + B.T)).max()
    assert top <= 1e-12 * scale
    if case == "far_field_box":
        assert top < -1e-4 * scale


@pytest.mark.parametrize("P,penalty,definite", [(2, 4.0, True), (3, 4.0, True), (2, 2.0, True), (2, 1.0, False),
                                               (3, 1.0, False)])
def test_stress_operator_is_symmetric(P, penalty, definite):
    """At rest, the BR2 momentum residual as a function of the velocity is the discrete
    div(tau(u)): symmetric in the quadrature inner product for any penalty, and negative
    semi-definite (like -int tau(u):grad u <= 0) only with a penalty of at least 2; with 1 the
    compressible stress operator has a growing mode for P >= 2."""
    mesh = W.periodic_rect_mesh(3, 3, 3.0, 3.0, jitter=0.15, seed=7)
    lev, lev0 = FRLevel(mesh, P, vgas(penalty=penalty)), FRLevel(mesh, P, vgas(mu=0.0))
    base = np.zeros((lev.ne, lev.npts, 4))
    base[..., 0], base[..., 3] = 100.0, 80.0
    blocks = [[_linear_operator(lev, lev0, base, vin, vout) for vin in (1, 2)] for vout in (1, 2)]
    A = np.block(blocks)
    wv = np.concatenate([weights(P, lev).reshape(-1)] * 2)
    B = wv[:, None] * A
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    top = np.linalg.eigvalsh(0.5 * (B + B.T)).max() / np.abs(B).max()
    assert (top <= 1e-12) if definite else (top > 1e-2)


def test_lifting_matches_its_dg_definition():
    """r_f of a face jump satisfies int_e r_f . tau = int_f tau (q_com - q) n_out dS for every
    tau of the element's polynomial space (the BR2 lifting), here with Lagrange basis tau."""
    mesh = W.periodic_rect_mesh(3, 3, 3.0, 3.0, jitter=0.15, seed=9)
    P = 3
    lev = FRLevel(mesh, P, vgas())
    n1, ne = lev.n1, lev.ne
    rng = np.random.default_rng(3)
    jump = rng.standard_normal((ne, 4, n1, 4))
    lift = lev.br2.liftings(jump)                               # [4, Ne, Np, 4, 2]
    wq = weights(P, lev)                                        # [Ne, Np]
    _, w1 = gauss_points(P)
    o = lev.ops
    for f in range(4):
        lhs = wq[:, :, None, None] * lift[f]                    # int r_f . e_m  per basis point m
        # face integral with the outward face vector: -N on the xi = -1 / eta = -1 faces
        sgn = -1.0 if f in (0, 2) else 1.0
        edge = o.lm if f in (0, 2) else o.lp
        rhs = np.zeros_like(lhs).reshape(ne, n1, n1, 4, 2)
        jn = sgn * jump[:, f, :, :, None] * lev.geo.fvec[:, f, :, None, :]   # [e, k, v, d]
        for k in range(n1):
            for m in range(n1):
                if f < 2:       # basis point (m, k): value on the face is l_m(+-1), face point k
                    rhs[:, k, m] += w1[k] * edge[m] * jn[:, k]
                else:           # basis point (k, m) on the eta line
                    rhs[:, m, k] += w1[k] * edge[m] * jn[:, k]
        assert np.abs(lhs - rhs.reshape(lhs.shape)).max() <= 1e-13 * np.abs(rhs).max()


def test_corrected_gradient_is_exact_for_linear_fields():
    """A field linear in (x, y) lies in every bilinear element's space and is continuous, so the
    jumps and liftings vanish and the corrected gradient is its exact gradient."""
    mesh = W.periodic_rect_mesh(4, 4, 4.0, 4.0, jitter=0.15, seed=1, ox=0.0, oy=0.0)
    lev = FRLevel(mesh, 2, vgas())
    x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
    a = np.array([1.0, 2.0, -1.0, 3.0])
    b = np.array([[0.5, -0.2], [1.0, 0.3], [-0.7, 0.1], [0.2, 0.9]])
    q = a + x[..., None] * b[:, 0] + y[..., None] * b[:, 1]
    g = lev.br2.local_gradient(q)
    assert np.abs(g - b[None, None]).max() <= 1e-12
    # away from the periodic seam the trace is continuous: zero jumps, zero liftings, and the
    # corrected gradient equals the exact one
    own = lev.traces(q)
    jump = 0.5 * (lev.outside_states(own, own) - own)
    gcor = g + lev.br2.liftings(jump).sum(axis=0)
    inner = [i + 4 * j for j in (1, 2) for i in (1, 2)]
    assert np.abs(jump[inner]).max() <= 1e-13
    assert np.abs(gcor[inner] - b[None, None]).max() <= 1e-12
    assert np.abs(gcor[0] - b[None]).max() > 1e-3         # a seam element sees its jumps


@pytest.mark.parametrize("P,min_rate", [(2, 0.8), (3, 1.7)])
def test_viscous_residual_is_consistent(P, min_rate):
    """R(mu) - R(0) against the exact div f_vis of a smooth periodic field (derivatives by the
    complex step and fourth-order differences) on jittered meshes 8 and 16 and 32: the
    pointwise error of a second-order operator falls like h^(P-1)."""
    L = 10.0
    kk = 2.0 * math.pi / L
    gas = G.Gas(gamma=1.4, rgas=1.0, eps_mode="local", mu=0.05)

    def field(x, y):
        return np.stack([100.0 + 0.5 * np.sin(kk * x) * np.cos(kk * y),
                         1.0 + 0.3 * np.sin(kk * x + 0.5) * np.sin(2 * kk * y),
                         0.5 + 0.2 * np.cos(2 * kk * x) * np.sin(kk * y),
                         80.0 + 0.4 * np.cos(kk * x - kk * y)], axis=-1)

    def flux(x, y, comp):
        h = 1e-30
        grad = np.stack([np.imag(field(x + 1j * h, y)) / h, np.imag(field(x, y + 1j * h)) / h], axis=-1)
        return viscous_flux(field(x, y), grad, gas)[comp]

    def exact_div(x, y, d=1e-3):
        c = [1 / 12, -2 / 3, 0.0, 2 / 3, -1 / 12]
        return (sum(cc * flux(x + (i - 2) * d, y, 0) for i, cc in enumerate(c))
                + sum(cc * flux(x, y + (i - 2) * d, 1) for i, cc in enumerate(c))) / d

    errs = []
    for n in (8, 16, 32):
        mesh = W.periodic_rect_mesh(n, n, L, L, jitter=0.1, seed=5, ox=0.0, oy=0.0)
        lev, lev0 = FRLevel(mesh, P, gas), FRLevel(mesh, P, G.Gas(gamma=1.4, rgas=1.0, eps_mode="local"))
        x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
        q = field(x, y)
        ex = exact_div(x, y)
        errs.append(np.abs(lev.residual(q) - lev0.residual(q) - ex).max() / np.abs(ex).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[0] > errs[1] > errs[2] and rates[-1] >= min_rate, (errs, rates)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_noslip_channel_conserves_mass_and_energy(P):
    """Periodic channel between no-slip adiabatic walls: nothing crosses the walls, so the
    quadrature sums of the mass and energy residuals vanish; the momentum sum (wall shear and
    pressure) does not."""
    mesh = W.channel_mesh(8, 4, 10.0, 2.0, jitter=0.1, seed=4)
    qinf = np.array([100.0 / 1.4, 1.0, 0.0, 100.0 / 1.4])
    lev = FRLevel(mesh, P, vgas(mu=0.05), q_inf=qinf)
    x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
    q = np.broadcast_to(qinf, x.shape + (4,)).copy()
    q[..., 0] += 0.5 * np.sin(0.6 * x) * np.cos(1.3 * y)
    q[..., 1] += 0.3 * np.sin(0.7 * x + 0.5) * np.sin(1.5 * y)
    q[..., 2] += 0.2 * np.cos(0.6 * x) * np.sin(1.1 * y)
    q[..., 3] += 0.4 * np.cos(0.9 * x)
    R = lev.residual(q)
    tot = np.einsum("ep,epv->v", weights(P, lev), R)
    mag = np.einsum("ep,epv->v", weights(P, lev), np.abs(R))
    assert abs(tot[0]) <= 1e-13 * mag[0] and abs(tot[3]) <= 1e-13 * mag[3]
    assert abs(tot[1]) > 1e-3 * mag[1]


def test_viscous_terms_vanish_for_uniform_flow():
    mesh = W.periodic_rect_mesh(4, 4, 4.0, 4.0, jitter=0.15, seed=1)
    q_inf = np.array([100.0, 1.0, 0.5, 80.0])
    lev, lev0 = FRLevel(mesh, 3, vgas(), q_inf=q_inf), FRLevel(mesh, 3, vgas(mu=0.0), q_inf=q_inf)
    q = np.broadcast_to(q_inf, (lev.ne, lev.npts, 4)).copy()
    # each term is (mu C_p / Pr) T / h^2 in size: rounding of the zero gradients only
    inv_h = np.max(np.linalg.norm(lev.geo.S_sp, axis=-1) / lev.geo.jac)
    scale = 0.3 * lev.gas.cp / lev.gas.prandtl * q_inf[3] * inv_h ** 2
    assert np.abs(lev.residual(q) - lev0.residual(q)).max() <= 1e-13 * scale


def test_viscous_element_block_matches_central_differences():
    mesh = W.channel_mesh(3, 3, 3.0, 3.0, jitter=0.1, seed=4)
    qinf = np.array([100.0 / 1.4, 1.0, 0.2, 100.0 / 1.4])
    lev = FRLevel(mesh, 2, vgas(mu=0.05), q_inf=qinf)
    x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
    q = np.broadcast_to(qinf, x.shape + (4,)).copy()
    q[..., 1] += 0.3 * np.sin(0.7 * x) * np.sin(1.5 * y)
    q[..., 3] += 0.4 * np.cos(0.9 * x + y)
    J = element_dFdq(lev, q)
    for e in (0, 4):                    # a wall element and an interior one
        Jfd = np.zeros((lev.n, lev.n))
        for c in range(lev.n):
            p, v = divmod(c, 4)
            h = 1e-4 * abs(q[e, p, v])
            qp, qm = q.copy(), q.copy()
            qp[e, p, v] += h
            qm[e, p, v] -= h
            Jfd[:, c] = (lev.residual(qp)[e] - lev.residual(qm)[e]).ravel() / (2 * h)
        colmax = np.max(np.abs(J[e]), axis=0)
        assert np.max(np.abs(Jfd - J[e]) / colmax) < 1e-6


def test_dtau_min_includes_the_viscous_limit():
    """eq. (33): with a large viscosity dtau_min = (dx/(P+1))^2 rho / mu."""
    mesh = W.periodic_quad_mesh(4, 10.0)
    q_inf = np.array([100.0, 0.6, 0.8, 100.0])
    gas = vgas(mu=50.0)
    sol = OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=(2,), n_smooth=(1,)), q_inf=q_inf)
    q = np.broadcast_to(q_inf, (16, 9, 4)).copy()
    h = 2.5 / 3
    assert abs(sol.dtau_min(q) - h * h * 1.0 / 50.0) <= 4e-15 * sol.dtau_min(q)
