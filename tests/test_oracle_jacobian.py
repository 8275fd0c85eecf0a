"""Pins of the oracle's element blocks D (Sec. 2.4, eqs. (28)-(30)) against central finite
differences of the global residual on tiny meshes."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle.fr import FRLevel
from oracle.jacobian import element_blocks, element_dFdq

GAS = G.Gas(eps_mode="local")


def _setup(P, n=3):
    mesh = W.periodic_quad_mesh(n, 10.0, jitter=0.1, seed=5)
    vs = W.VortexSpec(length=10.0)
    lev = FRLevel(mesh, P, GAS)
    q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
    return lev, q


@pytest.mark.parametrize("P", [1, 2])
def test_element_block_matches_central_differences(P):
    lev, q = _setup(P)
    c_mass = 1.0 / (0.29 * 0.05)
    J = element_dFdq(lev, q, c_mass)
    for e in (0, 4):
        Jfd = np.zeros((lev.n, lev.n))
        for c in range(lev.n):
            p, v = divmod(c, 4)
            h = 1e-4 * abs(q[e, p, v])      # central differences; the step balances h^2 and rounding
            qp, qm = q.copy(), q.copy()
            qp[e, p, v] += h
            qm[e, p, v] -= h
            Jfd[:, c] = (lev.stage_residual(qp, c_mass)[e] - lev.stage_residual(qm, c_mass)[e]).ravel() / (2 * h)
        colmax = np.max(np.abs(J[e]), axis=0)
        assert np.max(np.abs(Jfd - J[e]) / colmax) < 1e-6


def test_block_adds_gamma_over_dtau_and_mass_term():
    lev, q = _setup(1)
    dtau, c_mass = 0.7, 13.0
    D = element_blocks(lev, q, dtau, c_mass)
    D0 = element_blocks(lev, q, np.inf, 0.0)
    gam = G.preconditioner(q, GAS)
    M = G.mass_matrix(q, GAS)
    diff = D - D0
    for p in range(lev.npts):
        blk = diff[:, 4 * p:4 * p + 4, 4 * p:4 * p + 4]
        ref = gam[:, p] / dtau + c_mass * M[:, p]
        assert np.max(np.abs(blk - ref)) <= 1e-9 * np.max(np.abs(ref))
    off = diff.copy()
    for p in range(lev.npts):
        off[:, 4 * p:4 * p + 4, 4 * p:4 * p + 4] = 0
    assert np.max(np.abs(off)) <= 1e-9 * np.max(np.abs(diff))


def test_block_sparsity_is_line_structured():
    """A solution point couples only to points on its own xi- and eta-lines (tensor-product FR)."""
    lev, q = _setup(2)
    J = element_dFdq(lev, q)
    n1 = lev.n1
    for p in range(lev.npts):
        i, j = p % n1, p // n1
        for s in range(lev.npts):
            k, l = s % n1, s // n1
            blk = J[:, 4 * p:4 * p + 4, 4 * s:4 * s + 4]
            if k != i and l != j:
                assert np.max(np.abs(blk)) == 0.0


@pytest.mark.parametrize("case", ["periodic", "airfoil", "viscous"])
def test_patch_block_equals_whole_mesh_block(case):
    """The block of an element evaluated on its patch (the element and its face neighbours) equals
    the block from the whole mesh: the property the full-size GPU tests rely on to check sampled
    elements of meshes too large for the whole-mesh oracle blocks."""
    from patches import patch_block
    if case == "periodic":
        mesh = W.periodic_rect_mesh(7, 5, 10.0, 10.0, jitter=0.1, seed=3)
        gas, qinf, P = GAS, None, 2
        lev = FRLevel(mesh, P, gas)
        vs = W.VortexSpec(length=10.0)
        q = vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])
        picks = [0, 6, 17, 34]
    else:
        wall = W.BC_SLIP_WALL if case == "airfoil" else W.BC_NOSLIP_WALL
        mesh = W.airfoil_o_mesh(12, 4, ratio=1.3, r_far=6.0, wall=wall)
        fs = W.FreeStreamSpec(ma_inf=0.01)
        qinf = fs.freestream()
        gas = G.Gas(gamma=1.4, rgas=1.0, eps_mode="cutoff", ma_inf=0.01, kappa=1.0,
                    mu=(2e-3 if case == "viscous" else 0.0))
        P = 2
        lev = FRLevel(mesh, P, gas, q_inf=qinf)
        x, y = lev.geo.xy[..., 0], lev.geo.xy[..., 1]
        q = np.broadcast_to(qinf, x.shape + (4,)).copy()
        q[..., 0] += 0.5 * np.sin(0.7 * x) * np.cos(0.5 * y)
        q[..., 1] += 0.2 * np.cos(0.9 * x - 0.4 * y)
        q[..., 2] += 0.15 * np.sin(0.6 * y + 0.2 * x)
        picks = [0, 5, 11, 13, 40, 47]            # wall (incl. both trailing-edge sides), interior, far field
    full = element_blocks(lev, q, 0.3, 2.0)
    for e in picks:
        got = patch_block(mesh, gas, P, q, e, 0.3, 2.0, qinf)
        assert np.array_equal(got, full[e]) or np.max(np.abs(got - full[e])) <= 1e-13 * np.max(np.abs(full[e]))
