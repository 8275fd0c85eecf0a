"""Oracle pins for hexahedral levels (Sec. 2.3 in three dimensions, the sphere setting of
Sec. 4.2): the cubed-sphere mesh, the curl-form metric terms (exact for affine elements, discrete
metric identity, watertight faces), free-stream preservation on curved elements, discrete
conservation, spectral convergence of the residual to the exact flux divergence, element blocks
against central differences, and the 3-D transfers."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gas as OG
from oracle import solver as OS
from oracle.basis import Ops1D, gauss_points
from oracle.fr3 import FRLevel3, orient_map
from oracle.geometry3d import HexGeometry, element_dx3

FS = W.FreeStream3Spec(ma_inf=0.01)
GAS = OG.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=0.01, kappa=1.0)


def rotated(mesh, elems, inner):
    """The mesh with the local node numbering of the given elements rotated (quarter turns about
    zeta and about xi), so that their faces meet neighbours with swapped and reversed point
    orders; connectivity rebuilt (boundary faces found again by their radius)."""
    nodes = mesh.nodes.copy()
    c, b, a = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    new = a + 3 * b + 9 * c
    rot_z = (2 - b) + 3 * a + 9 * c          # new (a, b, c) takes the old node (2 - b, a, c)
    rot_x = a + 3 * (2 - c) + 9 * b          # new (a, b, c) takes the old node (a, 2 - c, b)
    for t, e in enumerate(elems):            # element t: (t % 4) turns about zeta, (t // 4 % 3) about xi
        for perm in [rot_z] * (t % 4) + [rot_x] * (t // 4 % 3):
            y = np.empty_like(nodes[e])
            y[new] = nodes[e][perm]
            nodes[e] = y
    r = np.linalg.norm(nodes, axis=-1)
    rin, rout = r.min(), r.max()

    def tag(e, f):
        rc = np.linalg.norm(nodes[e, (12, 14, 10, 16, 4, 22)[f]])
        if abs(rc - rout) < 1e-9 * rout:
            return W.BC_FAR_FIELD
        if abs(rc - rin) < 1e-9:
            return inner
        raise ValueError("unmatched interior face")

    nbr, nbf, ori = W.connect_hex_mesh(nodes, tag)
    return W.Mesh(3, 2, nodes, nbr, nbf, ori, name=mesh.name + "_rot")


def small_sphere(inner=W.BC_FAR_FIELD, rotate=True, shells=2):
    m = W.cubed_sphere_mesh(3, shells, ratio=1.3, r_far=4.0, inner=inner)
    return rotated(m, [0, 5, 11, 20, 33, 47, 58, 64, 70, 77, 83, 90, 97, 101], inner) if rotate else m


def test_cubed_sphere_mesh():
    mesh = W.cubed_sphere_mesh(4, 3)
    ne = mesh.n_elements
    assert ne == 6 * 16 * 3
    e = np.arange(ne)
    for f in range(6):
        nb = mesh.face_nbr[:, f]
        ok = nb >= 0
        assert np.all(mesh.face_nbr[nb[ok], mesh.face_nbr_face[ok, f]] == e[ok])
    assert np.sum(mesh.face_nbr[:, 4] == W.BC_SLIP_WALL) == 96
    assert np.sum(mesh.face_nbr[:, 5] == W.BC_FAR_FIELD) == 96
    r = np.linalg.norm(mesh.nodes, axis=-1)
    assert abs(r.min() - 1.0) < 1e-14 and abs(r.max() - 20.0) < 1e-13
    rot = small_sphere()
    assert len(np.unique(rot.face_orient)) >= 4          # swapped and reversed faces occur


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_full_mesh_jacobian_positive_and_volume(P):
    """|J| > 0 at every solution point of the 6 x 16 x 16 x 24 sphere mesh; with P = 3 the volume
    matches the spherical shell to the quadratic geometry's accuracy."""
    mesh, _ = W.sphere_config5()
    geo = HexGeometry(mesh, P)
    assert np.all(geo.jac > 0.0)
    if P == 3:
        _, w = gauss_points(P)
        ww = np.einsum("k,j,i->kji", w, w, w).ravel()
        vol = np.sum(geo.jac * ww[None, :])
        exact = 4.0 / 3.0 * math.pi * (20.0 ** 3 - 1.0)
        assert abs(vol - exact) < 2e-4 * exact


def test_metrics_exact_on_affine_elements():
    """For an affine map the curl form reproduces the exact constant metric vectors."""
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.9, 0.3], [-0.2, 0.15, 1.1]])
    c, b, a = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    ref = np.stack([a.ravel() - 1.0, b.ravel() - 1.0, c.ravel() - 1.0], axis=-1)   # node a + 3b + 9c
    tags = -2 * np.ones((1, 6), np.int32)
    lin = W.Mesh(3, 2, (ref @ A.T)[None], tags, np.zeros((1, 6), np.int32), np.zeros((1, 6), np.int32))
    J = np.linalg.det(A)
    cof = J * np.linalg.inv(A)                                    # row d: J grad xi^d
    for P in (1, 2, 3):
        g = HexGeometry(lin, P)
        for d in range(3):
            assert np.max(np.abs(g.Ja[:, d] - cof[d])) < 1e-13
        assert np.max(np.abs(g.jac - J)) < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3])
def test_discrete_metric_identity_and_watertight_faces(P):
    mesh = small_sphere()
    g = HexGeometry(mesh, P)
    o = Ops1D(P)
    n1 = P + 1
    ne = mesh.n_elements
    div = np.zeros((ne, n1, n1, n1, 3))
    for d, (sub) in enumerate(("im,ekjmn->ekjin", "jm,ekmin->ekjin", "km,emjin->ekjin")):
        div += np.einsum(sub, o.D, g.Ja[:, d].reshape(ne, n1, n1, n1, 3))
    scale = np.max(np.abs(g.Ja))
    assert np.max(np.abs(div)) < 1e-13 * scale
    for e in range(ne):
        for f in range(6):
            nb = mesh.face_nbr[e, f]
            if nb < 0:
                continue
            nf = mesh.face_nbr_face[e, f]
            sign = 1.0 if (f % 2) != (nf % 2) else -1.0
            theirs = g.fvec[nb, nf][orient_map(mesh.face_orient[e, f], n1)]
            assert np.max(np.abs(g.fvec[e, f] - sign * theirs)) < 1e-13 * scale


@pytest.mark.parametrize("P", [1, 2, 3])
def test_freestream_preserved_on_curved_hexes(P):
    mesh = small_sphere()
    lev = FRLevel3(mesh, P, GAS, q_inf=FS.freestream())
    qinf = np.array([FS.freestream()[0], 0.6, -0.48, 0.64, FS.freestream()[4]])
    lev.q_inf = qinf
    q = np.broadcast_to(qinf, (mesh.n_elements, lev.npts, 5)).copy()
    R = lev.residual(q)
    inv_h = np.max(np.linalg.norm(lev.geo.Ja, axis=-1) / lev.geo.jac[:, None, :])
    scale = qinf[0] * inv_h
    assert np.max(np.abs(R[..., :4])) / scale < 1e-13
    assert np.max(np.abs(R[..., 4])) / scale < 1e-13 / 0.01 ** 2


@pytest.mark.parametrize("P", [1, 2])
def test_discrete_conservation(P):
    """sum over elements and points of w |J| R equals minus the common flux through the boundary
    faces integrated with the face rule (interior face fluxes cancel)."""
    mesh = small_sphere()
    lev = FRLevel3(mesh, P, GAS, q_inf=FS.freestream())
    x = lev.geo.xyz
    q = np.broadcast_to(FS.freestream(), x.shape[:2] + (5,)).copy()
    q[..., 0] *= 1.0 + 1e-3 * np.sin(x[..., 0]) * np.cos(0.7 * x[..., 1])
    q[..., 1] += 0.2 * np.cos(0.5 * x[..., 2])
    q[..., 3] += 0.1 * np.sin(0.3 * x[..., 0] + 0.2 * x[..., 1])
    R = lev.residual(q)
    _, w = gauss_points(P)
    ww = np.einsum("k,j,i->kji", w, w, w).ravel()
    total = np.einsum("ep,p,epv->v", lev.geo.jac, ww, R)
    own = lev.traces(q)
    out = lev.outside_states(own, own)
    wf = np.outer(w, w).ravel()                    # weight of face point k1 + n1 k2 is w_k1 w_k2
    bsum = np.zeros(5)
    for f in range(6):
        bnd = mesh.face_nbr[:, f] < 0
        fv = lev.geo.fvec[bnd, f]
        if f % 2 == 0:                              # +xi^d points into the element: outward = -
            fh = -OG.common_flux(out[bnd, f], own[bnd, f], fv, GAS)
        else:
            fh = OG.common_flux(own[bnd, f], out[bnd, f], fv, GAS)
        bsum += np.einsum("k,ekv->v", wf, fh)
    scale = np.max(np.abs(np.einsum("ep,p,epv->epv", lev.geo.jac, ww, R)))
    assert np.max(np.abs(total + bsum)) < 1e-11 * scale


def test_residual_converges_to_flux_divergence():
    """R of a smooth field approaches -div f of the exact field as P grows (curved elements)."""
    mesh = small_sphere(shells=3)
    errs = []
    for P in (1, 2, 3, 4):
        lev = FRLevel3(mesh, P, GAS, q_inf=FS.freestream())
        x = lev.geo.xyz

        def field(xx):
            q = np.zeros(xx.shape[:-1] + (5,), dtype=xx.dtype)
            q[..., 0] = FS.freestream()[0] * (1.0 + 0.01 * np.sin(0.5 * xx[..., 0]) * np.cos(0.4 * xx[..., 1]))
            q[..., 1] = 1.0 + 0.3 * np.sin(0.4 * xx[..., 2])
            q[..., 2] = 0.2 * np.cos(0.3 * xx[..., 0])
            q[..., 3] = 0.1 * np.sin(0.5 * xx[..., 1])
            q[..., 4] = FS.freestream()[4] * (1.0 + 0.01 * np.cos(0.3 * xx[..., 2]))
            return q

        q = field(x)
        R = lev.residual(q)             # compared on the elements without a boundary face
        h = 1e-30
        exact = np.zeros_like(R)
        for n in range(3):
            xc = x.astype(complex)
            xc[..., n] += 1j * h
            unit = np.zeros(3)
            unit[n] = 1.0
            exact -= OG.normal_flux(field(xc), unit, GAS).imag / h
        interior = np.all(mesh.face_nbr >= 0, axis=1)
        err = np.max(np.abs(R[interior] - exact[interior]), axis=(0, 1)) / np.max(np.abs(exact[interior]), axis=(0, 1))
        errs.append(err[1])
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1] and errs[3] < 0.3 * errs[2], errs


def test_element_block_matches_central_differences():
    from oracle.jacobian import element_dFdq
    mesh = small_sphere(inner=W.BC_SLIP_WALL)
    lev = FRLevel3(mesh, 1, GAS, q_inf=FS.freestream())
    x = lev.geo.xyz
    q = np.broadcast_to(FS.freestream(), x.shape[:2] + (5,)).copy()
    q[..., 0] *= 1.0 + 1e-3 * np.sin(x[..., 0])
    q[..., 1] += 0.2 * np.cos(0.5 * x[..., 2])
    q[..., 2] += 0.1 * np.sin(0.4 * x[..., 1])
    c_mass = 3.0
    J = element_dFdq(lev, q, c_mass)
    for e in (0, 40):                               # a wall element, an outer one
        Jfd = np.zeros((lev.n, lev.n))
        for c in range(lev.n):
            p, v = divmod(c, 5)
            hh = 1e-4 * max(abs(q[e, p, v]), 0.1)
            qp, qm = q.copy(), q.copy()
            qp[e, p, v] += hh
            qm[e, p, v] -= hh
            Jfd[:, c] = (lev.stage_residual(qp, c_mass)[e] - lev.stage_residual(qm, c_mass)[e]).ravel() / (2 * hh)
        colmax = np.max(np.abs(J[e]), axis=0)
        assert np.max(np.abs(Jfd - J[e]) / colmax) < 1e-6


def test_transfers_3d():
    """3-D restriction then prolongation is the identity on the coarse space and exact on
    polynomials of the coarse degree."""
    rng = np.random.default_rng(3)
    for Pf, Pc in ((2, 1), (1, 0), (3, 2)):
        xc = rng.standard_normal((4, (Pc + 1) ** 3, 5))
        xf = OS.prolong(xc, Pc, Pf, dim=3)
        assert np.max(np.abs(OS.restrict(xf, Pf, Pc, dim=3) - xc)) < 1e-13


def test_element_dx3_closed_form():
    """Delta x on an axis-aligned box of sides (2, 3, 5): twice the centroid's distance to the
    nearest face, i.e. the smallest side."""
    nodes = np.stack(np.meshgrid([0.0, 1.0, 2.0], [0.0, 1.5, 3.0], [0.0, 2.5, 5.0], indexing="ij"), -1)
    nodes = nodes.transpose(2, 1, 0, 3).reshape(1, 27, 3)
    m = W.Mesh(3, 2, nodes, -2 * np.ones((1, 6), np.int32), np.zeros((1, 6), np.int32), np.zeros((1, 6), np.int32))
    assert abs(element_dx3(m)[0] - 2.0) < 1e-13
