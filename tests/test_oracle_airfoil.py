"""Oracle pins for the curved-wall configuration (Sec. 4.2): the 9-node O-mesh, free-stream
preservation on curved elements, the slip-wall flux, and the CFL pseudo-time scale of
eqs. (32)-(33)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.fr import FRLevel
from oracle.geometry import QuadGeometry, element_dx

FS = W.FreeStreamSpec()


def cutoff_gas(ma=FS.ma_inf):
    return OG.Gas(gamma=FS.gamma, rgas=FS.rgas, eps_mode="cutoff", ma_inf=ma, kappa=1.0)


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_o_mesh_mapping_is_valid(P):
    """|J| > 0 at every solution point of the full 128 x 64 O-mesh, and the elements tile the
    region between the profile and the far-field circle (total area = circle - profile)."""
    mesh = W.airfoil_o_mesh(128, 64)
    geo = QuadGeometry(mesh, P)
    assert np.all(geo.jac > 0.0)
    if P == 4:
        from oracle.basis import gauss_points
        _, w = gauss_points(P)
        ww = np.outer(w, w).ravel()
        area = np.sum(geo.jac * ww[None, :])
        # profile area of the closed 12% section: integral of 2 y_t over the chord (fine trapezoid rule)
        x = 0.5 * (1.0 - np.cos(np.linspace(0.0, np.pi, 200001)))
        yt = W.naca4_symmetric_half_thickness(x, 0.12)
        prof = np.sum(np.diff(x) * (yt[1:] + yt[:-1]))
        # the quadratic elements interpolate the far-field circle and the profile by parabolas,
        # which changes the area by O((2 pi / 128)^4) relative (1.5e-5 absolute here)
        assert abs(area - (math.pi * 20.0 ** 2 - prof)) < 1e-7 * math.pi * 400.0


def test_o_mesh_connectivity():
    mesh = W.airfoil_o_mesh(16, 6)
    nw = 16
    for e in range(mesh.n_elements):
        i, j = e % nw, e // nw
        for f in range(4):
            nb = mesh.face_nbr[e, f]
            if nb >= 0:
                assert mesh.face_nbr[nb, mesh.face_nbr_face[e, f]] == e
                # shared corner nodes coincide
                a = {0: (0, 6), 1: (2, 8), 2: (0, 2), 3: (6, 8)}
                ca = mesh.nodes[e, list(a[f])]
                cb = mesh.nodes[nb, list(a[mesh.face_nbr_face[e, f]])]
                assert np.allclose(ca, cb, atol=1e-13)
        assert (mesh.face_nbr[e, 2] == W.BC_SLIP_WALL) == (j == 0)
        assert (mesh.face_nbr[e, 3] == W.BC_FAR_FIELD) == (j == 5)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_freestream_preserved_on_curved_annulus(P):
    """A uniform flow is an exact steady solution; on quadratic elements with metrics from the
    exact mapping the FR residual keeps it to rounding (far field on both boundaries)."""
    mesh = W.airfoil_o_mesh(32, 16, annulus=True, r_far=5.0)
    gas = cutoff_gas()
    qinf = FS.freestream()
    lev = FRLevel(mesh, P, gas, q_inf=qinf)
    q = np.broadcast_to(qinf, lev.geo.xy.shape[:2] + (4,)).copy()
    R = lev.residual(q)
    inv_h = np.max(np.linalg.norm(lev.geo.S_sp, axis=-1) / lev.geo.jac)
    rho = qinf[0] / (FS.rgas * qinf[3])
    scale = qinf[0] * 1.0 * inv_h
    escale = rho * float(OG.total_enthalpy(qinf, gas)) * 1.0 * inv_h
    assert np.max(np.abs(R[..., :3])) / scale < 1e-13
    # the preconditioned dissipation amplifies pressure rounding by 1/eps^2 = 1/Ma^2 in energy
    assert np.max(np.abs(R[..., 3])) / escale < 1e-13 / FS.ma_inf ** 2


@pytest.mark.parametrize("eps_mode,ma", [("local", 0.005), ("cutoff", 0.001)])
def test_slip_wall_flux_is_impermeable(eps_mode, ma):
    """With the mirrored ghost state the common flux of eq. (21) carries no mass or energy through
    the wall and its momentum part is normal to the wall (a pressure force)."""
    gas = OG.Gas(gamma=1.4, rgas=1.0, eps_mode=eps_mode, ma_inf=ma, kappa=1.0)
    rng = np.random.default_rng(5)
    for _ in range(16):
        t = (1.0 / ma) ** 2 / 1.4 * (1.0 + 0.01 * rng.standard_normal())
        p = t * (1.0 + 0.01 * rng.standard_normal())
        u = rng.standard_normal(2)
        th = rng.uniform(0.0, 2.0 * np.pi)
        n = np.array([math.cos(th), math.sin(th)])
        q = np.array([p, u[0], u[1], t])
        ghost = q.copy()
        ghost[1:3] = u - 2.0 * (u @ n) * n
        s = 1.7 * n
        f = OG.common_flux(q, ghost, s, gas)
        scale = 1.7 * p
        assert abs(f[0]) / scale < 1e-14
        assert abs(f[3]) / (scale * np.linalg.norm(u)) < 1e-13
        assert abs(f[1] * n[1] - f[2] * n[0]) / scale < 1e-14
        # and the wall pressure force is close to p (it is p plus an acoustic correction)
        assert abs((f[1] * n[0] + f[2] * n[1]) / 1.7 - p) / p < 1e-3


def test_element_dx_closed_forms():
    """Delta x of eq. (33): min(width, height) on rectangles; on an isosceles trapezoid, twice the
    distance from the centroid (height h (a + 2b) / (3 (a + b))) to its nearest side."""
    mesh = W.periodic_rect_mesh(5, 3, 10.0, 3.0)
    assert np.allclose(element_dx(mesh), 1.0, rtol=1e-14, atol=0)
    mesh = W.periodic_rect_mesh(4, 4, 2.0, 8.0)
    assert np.allclose(element_dx(mesh), 0.5, rtol=1e-14, atol=0)
    a, b, h = 3.0, 1.0, 2.0                     # bottom, top, height
    corners = np.array([[-a / 2, 0.0], [a / 2, 0.0], [-b / 2, h], [b / 2, h]])
    nodes = corners[None]                       # bilinear element, node a + 2 b
    mesh = W.Mesh(2, 1, nodes, -np.ones((1, 4), np.int32), np.zeros((1, 4), np.int32),
                  np.zeros((1, 4), np.int32))
    yc = h * (a + 2 * b) / (3 * (a + b))
    # distance from (0, yc) to the line through (a/2, 0) and (b/2, h)
    px, py, dx, dy = a / 2, 0.0, (b - a) / 2, h
    d_side = abs(dx * (yc - py) - dy * (0.0 - px)) / math.hypot(dx, dy)
    expect = 2.0 * min(yc, h - yc, d_side)
    assert abs(element_dx(mesh)[0] - expect) < 1e-14 * expect


def test_dtau_min_uniform_state():
    """eq. (33) on a uniform mesh and state: dtau_min = (dx/(P+1)) / (c + |v|) exactly."""
    mesh = W.periodic_quad_mesh(4, 10.0)
    gas = cutoff_gas(0.01)
    q_inf = np.array([1.0 / 0.01 ** 2 / 1.4, 0.6, 0.8, 1.0 / 0.01 ** 2 / 1.4])
    sol = OS.PMGSolver(mesh, gas, OS.PMGOptions(p_levels=(3, 1), n_smooth=(1, 1)), q_inf=q_inf)
    q = np.broadcast_to(q_inf, (16, 16, 4)).copy()
    c = math.sqrt(1.4 * q_inf[3])
    assert abs(sol.dtau_min(q) - (2.5 / 4) / (c + 1.0)) < 1e-15 * sol.dtau_min(q)


def test_cfl_stage_solve_scales_pseudo_time():
    """With the CFL form the stage solve starts at cfl_init * dtau_min and the SER law caps the
    step at cfl_max * dtau_min; a steady airfoil solve from the free stream drops the residual."""
    mesh = W.airfoil_o_mesh(12, 4, ratio=1.3, r_far=6.0)
    gas = cutoff_gas()
    qinf = FS.freestream()
    opts = OS.PMGOptions(p_levels=(2, 1), n_smooth=(3, 6), use_cfl=True, cfl_init=1e2, cfl_max=1e5,
                         max_vcycles=12, tol=1e-30)
    sol = OS.PMGSolver(mesh, gas, opts, q_inf=qinf)
    q0 = np.broadcast_to(qinf, (mesh.n_elements, 9, 4)).copy()
    dmin = sol.dtau_min(q0)
    _, st = sol.stage_solve(q0)
    assert st.dtau_scale == (1e2 * dmin, 1e5 * dmin)
    assert st.dtau_history[0] == 1e2 * dmin
    assert max(st.dtau_history) <= 1e5 * dmin
    assert st.history[-1] < 0.1 * st.history[0]


def test_wall_element_block_matches_central_differences():
    """The element block of a slip-wall element against central differences of the residual
    (the wall ghost depends on the element's own trace)."""
    from oracle.jacobian import element_dFdq
    mesh = W.airfoil_o_mesh(8, 3, ratio=1.3, r_far=6.0)
    gas = cutoff_gas()
    qinf = FS.freestream()
    lev = FRLevel(mesh, 2, gas, q_inf=qinf)
    x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
    q = np.broadcast_to(qinf, x.shape + (4,)).copy()
    q[..., 0] += 0.8 * np.sin(0.7 * x) * np.cos(0.5 * y)
    q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
    q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
    J = element_dFdq(lev, q)
    for e in (1, 13):                   # a wall element (j = 0) and one of the next layer
        assert (mesh.face_nbr[e, 2] == W.BC_SLIP_WALL) == (e < 8)
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
