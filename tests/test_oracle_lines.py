"""Pins of the oracle's element-line Jacobi (``oracle.lines``): its neighbour blocks against
the complex-step Jacobian of the whole residual, its line solve against a block-Thomas
recursion, and its reduction to element Jacobi (eq. (30)) for lines of one element."""
import numpy as np
import pytest

import workloads as W
from oracle import gas as G
from oracle import lines as OL
from oracle.fr import FRLevel
from oracle.jacobian import H_STEP, element_blocks, element_dFdq

FS = W.FreeStreamSpec()


def airfoil_case(P, nw=6, nr=4, seed=3):
    """A small O-mesh around the profile (wall, far field, periodic wrap) at a disturbed free
    stream, so that every block is non-trivial."""
    mesh = W.airfoil_o_mesh(nw, nr)
    gas = G.Gas(gamma=FS.gamma, rgas=FS.rgas, eps_mode="cutoff", ma_inf=FS.ma_inf, kappa=1.0)
    q_inf = FS.freestream()
    lev = FRLevel(mesh, P, gas, q_inf)
    rng = np.random.default_rng(seed)
    q = np.broadcast_to(q_inf, (lev.ne, lev.npts, 4)).copy()
    q[..., 0] *= 1.0 + 1e-6 * rng.standard_normal(q.shape[:2])
    q[..., 1:3] += 0.05 * rng.standard_normal(q.shape[:2] + (2,))
    q[..., 3] *= 1.0 + 1e-6 * rng.standard_normal(q.shape[:2])
    return lev, q


def vortex_case(P):
    mesh = W.periodic_quad_mesh(3, 10.0, jitter=0.1, seed=5)
    vs = W.VortexSpec(length=10.0)
    lev = FRLevel(mesh, P, G.Gas(eps_mode="local"))
    return lev, vs.state(lev.geo.xy[..., 0], lev.geo.xy[..., 1])


def radial_lines(nw, nr):
    """The O-mesh's radial lines, wall to far field: element i + nw j for j = 0 .. nr-1."""
    return np.arange(nw)[:, None] + nw * np.arange(nr)[None, :]


@pytest.mark.parametrize("case", ["airfoil_P1", "airfoil_P2", "vortex_P2"])
def test_neighbour_blocks_are_the_off_diagonal_jacobian(case):
    """Brute force: the complex-step derivative of the whole residual with respect to one
    unknown of element e' is, on e', column c of dR_e'/dq_e'; on each neighbour e across its
    face f, column c of -A_{e,e'} = -neighbour_blocks(f)[e]; zero elsewhere."""
    kind, P = case.split("_P")
    lev, q = airfoil_case(int(P)) if kind == "airfoil" else vortex_case(int(P))
    mesh = lev.mesh
    nb = [OL.neighbour_blocks(lev, q, f) for f in range(4)]
    J = element_dFdq(lev, q)
    scale = max(np.max(np.abs(J)), max(np.max(np.abs(b)) for b in nb))
    rng = np.random.default_rng(7)
    for e1 in rng.choice(lev.ne, 3, replace=False):
        for c in rng.choice(lev.n, 3, replace=False):
            p, v = divmod(int(c), 4)
            qc = q.astype(complex)
            qc[e1, p, v] += 1j * H_STEP
            col = lev.residual(qc).imag.reshape(lev.ne, lev.n) / H_STEP
            expect = np.zeros_like(col)
            expect[e1] = J[e1][:, c]
            for f in range(4):
                e = int(mesh.face_nbr[e1, f])
                if e >= 0:
                    expect[e] += -nb[mesh.face_nbr_face[e1, f]][e][:, c]
            assert np.max(np.abs(col - expect)) < 1e-12 * scale


def test_neighbour_blocks_vanish_on_boundary_faces_and_are_line_sparse():
    """The wall face of the first layer and the far-field face of the last carry no neighbour
    block; an interior block couples a point only to the neighbour's points on the matching
    line through the shared face (Nv (P+1) nonzero columns per row)."""
    P = 2
    lev, q = airfoil_case(P)
    nw = 6
    A2 = OL.neighbour_blocks(lev, q, 2)
    A3 = OL.neighbour_blocks(lev, q, 3)
    assert np.all(A2[:nw] == 0.0) and np.all(A3[-nw:] == 0.0)
    nz = np.count_nonzero(np.abs(A3[nw]) > 0.0, axis=1)
    assert np.all(nz <= 4 * (P + 1)) and np.max(nz) > 0


def test_line_solve_is_the_block_thomas_recursion():
    """The dense solve of the block-tridiagonal line matrix equals the block-Thomas recursion
    D'_k = D_k - Am_k D'_{k-1}^{-1} Ap_{k-1}, y_k = D'_k^{-1}(b_k - Am_k y_{k-1}),
    x_k = y_k - D'_k^{-1} Ap_k x_{k+1}."""
    rng = np.random.default_rng(11)
    K, n = 6, 9
    D = rng.standard_normal((K, n, n)) + 8.0 * np.eye(n)
    Am = rng.standard_normal((K, n, n))
    Ap = rng.standard_normal((K, n, n))
    line = np.arange(K)
    b = rng.standard_normal((K, n))
    Wi, y = [], []
    for k in range(K):
        Dk = D[k] - (Am[k] @ Wi[k - 1] @ Ap[k - 1] if k else 0.0)
        Wi.append(np.linalg.inv(Dk))
        y.append(Wi[k] @ (b[k] - (Am[k] @ y[k - 1] if k else 0.0)))
    x = [None] * K
    for k in reversed(range(K)):
        x[k] = y[k] - (Wi[k] @ Ap[k] @ x[k + 1] if k + 1 < K else 0.0)
    assert np.allclose(OL.line_solve(D, Am, Ap, line, b), np.array(x), rtol=1e-12, atol=1e-12)


def test_lines_of_one_element_are_element_jacobi():
    """With lines of length one every coupling is dropped: one line sweep is one element-Jacobi
    sweep of eq. (30)."""
    lev, q = airfoil_case(1)
    dtau, c_mass = 0.3, 2.0
    lines = np.arange(lev.ne)[:, None]
    blocks = OL.line_blocks(lev, q, dtau, c_mass, lines)
    assert np.all(blocks[1] == 0.0) and np.all(blocks[2] == 0.0)
    S = 0.01 * lev.stage_residual(q, c_mass)
    q1 = OL.line_sweeps(lev, q, blocks, lines, 1, c_mass, None, S)
    D = element_blocks(lev, q, dtau, c_mass)
    F = lev.stage_residual(q, c_mass, None, S).reshape(lev.ne, lev.n, 1)
    q2 = q + np.linalg.solve(D, F).reshape(q.shape)
    assert np.max(np.abs(q1 - q2)) <= 1e-12 * np.max(np.abs(q2 - q))


def test_line_blocks_follow_the_line_order():
    """Am of a line's first element and Ap of its last are zero; inside the line Am[e] is the
    block towards the previous element and Ap[e] towards the next, whatever the direction in
    which the line runs."""
    lev, q = airfoil_case(1)
    nw, nr = 6, 4
    lines = radial_lines(nw, nr)
    D, Am, Ap = OL.line_blocks(lev, q, 0.5, 0.0, lines)
    rev = lines[:, ::-1].copy()
    D2, Am2, Ap2 = OL.line_blocks(lev, q, 0.5, 0.0, rev)
    assert np.all(Am[lines[:, 0]] == 0.0) and np.all(Ap[lines[:, -1]] == 0.0)
    assert np.array_equal(Am, Ap2) and np.array_equal(Ap, Am2) and np.array_equal(D, D2)
    A3 = OL.neighbour_blocks(lev, q, 3)
    assert np.array_equal(Ap[lines[:, 1]], A3[lines[:, 1]])


def test_check_lines_rejects_bad_lines():
    lev, _ = airfoil_case(0)
    with pytest.raises(ValueError):
        OL.check_lines(lev.mesh, np.arange(lev.ne).reshape(2, -1))       # wrap rows: not neighbours at the seam
    with pytest.raises(ValueError):
        OL.check_lines(lev.mesh, np.zeros((lev.ne, 1), int))
