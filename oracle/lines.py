"""Element-line Jacobi: the block-tridiagonal smoother along lines of elements.

The pseudo-transient linearisation of a stage (eq. (28)) is A = Gamma/dtau - dF/dq.
Element Jacobi (eq. (30)) keeps only its diagonal blocks D_e. Line Jacobi is the remedy the
introduction cites from prior implicit high-order work for the stiffness that strong mesh
stretching brings. It keeps two more blocks for each element on a line of face-connected
elements (an O-mesh's radial lines, say): the blocks that couple it to its predecessor and its
successor,

    A_{e,e'} = -dF_e/dq_{e'} = -dR_e/dq_{e'}.

A neighbour enters R_e only through the common flux on the shared face (eq. (21)). The
mass and source terms of F are element-local. The smoother solves the block-tridiagonal
system of every line exactly and treats the lines independently (Jacobi across lines):

    q <- q + alpha_r A_line^{-1} (F(q) - S)

The couplings to neighbours outside the line are dropped, as element Jacobi drops all of
them. With lines of one element the sweep is element Jacobi.

The neighbour blocks are complex-step derivatives, as the diagonal blocks in
``oracle.jacobian`` are. The line solve is the plain definition: the dense
block-tridiagonal matrix of the line and a LAPACK solve.

This module is test infrastructure. Only the tests, the smoke entry point and the
benchmark's CPU baseline may use it.
"""
from __future__ import annotations

import numpy as np

from .jacobian import H_STEP, element_blocks


def face_towards(mesh, e: int, e2: int) -> int:
    """The face of element e whose neighbour is e2 (exactly one such face is required)."""
    faces = [f for f in range(mesh.face_nbr.shape[1]) if int(mesh.face_nbr[e, f]) == e2]
    if len(faces) != 1:
        raise ValueError(f"elements {e} and {e2} do not share exactly one face")
    return faces[0]


def check_lines(mesh, lines) -> np.ndarray:
    """lines [n_lines, K] of element indices: every element exactly once, consecutive entries
    face neighbours."""
    lines = np.asarray(lines, dtype=np.int64)
    if lines.ndim != 2 or lines.size != mesh.n_elements:
        raise ValueError("lines must be a [n_lines, K] array covering every element")
    if not np.array_equal(np.sort(lines.ravel()), np.arange(mesh.n_elements)):
        raise ValueError("every element must appear on exactly one line")
    for line in lines:
        for k in range(len(line) - 1):
            face_towards(mesh, int(line[k]), int(line[k + 1]))
    return lines


def neighbour_blocks(level, q, f: int) -> np.ndarray:
    """A_{e, nb(e,f)} = -dR_e/dq_{nb(e,f)} for every element e across its face f, [Ne, n, n]
    (index p*Nv + v on both sides). A block is zero where face f is a boundary.

    Column c perturbs unknown c of every element at once, with the complex step. Only face f of
    each element sees the perturbed neighbour state, so element e responds to its one
    neighbour across f.
    """
    ne, npts, nv = q.shape
    n = npts * nv
    qr = np.asarray(q, float)
    out = np.zeros((ne, n, n))
    for c in range(n):
        p, v = divmod(c, nv)
        qc = qr.astype(complex)
        qc[:, p, v] += 1j * H_STEP
        R = level.residual(qr, q_nbr=qc, nbr_faces=(f,))
        out[:, :, c] = -R.imag.reshape(ne, n) / H_STEP
    out[level.mesh.face_nbr[:, f] < 0] = 0.0
    return out


def line_blocks(level, q, dtau, c_mass, lines):
    """D_e (eqs. (28), (30)) and, per element, Am[e] = A_{e, previous on its line} and
    Ap[e] = A_{e, next on its line} (zero at the line's ends), each [Ne, n, n]."""
    mesh = level.mesh
    lines = check_lines(mesh, lines)
    D = element_blocks(level, q, dtau, c_mass)
    nb = [None] * mesh.face_nbr.shape[1]
    Am = np.zeros_like(D)
    Ap = np.zeros_like(D)
    for line in lines:
        for k, e in enumerate(line):
            for other, dst in ((k - 1, Am), (k + 1, Ap)):
                if 0 <= other < len(line):
                    f = face_towards(mesh, int(e), int(line[other]))
                    if nb[f] is None:
                        nb[f] = neighbour_blocks(level, q, f)
                    dst[e] = nb[f][e]
    return D, Am, Ap


def line_matrix(D, Am, Ap, line) -> np.ndarray:
    """The dense block-tridiagonal matrix of one line: block (k, k) = D, (k, k-1) = Am,
    (k, k+1) = Ap of the line's k-th element."""
    K, n = len(line), D.shape[1]
    M = np.zeros((K * n, K * n))
    for k, e in enumerate(line):
        M[k * n:(k + 1) * n, k * n:(k + 1) * n] = D[e]
        if k > 0:
            M[k * n:(k + 1) * n, (k - 1) * n:k * n] = Am[e]
        if k + 1 < K:
            M[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = Ap[e]
    return M


def line_solve(D, Am, Ap, line, b) -> np.ndarray:
    """x with A_line x = b for one line; b and x are [K, n]."""
    K, n = len(line), D.shape[1]
    x = np.linalg.solve(line_matrix(D, Am, Ap, line), np.asarray(b).reshape(K * n))
    return x.reshape(K, n)


def line_sweeps(level, q, blocks, lines, nsweep, c_mass=0.0, src=None, S=None, alpha_r=1.0):
    """nsweep line-Jacobi sweeps: q <- q + alpha_r A_line^{-1} (F(q) - S) on every line at once."""
    D, Am, Ap = blocks
    lines = np.asarray(lines, dtype=np.int64)
    ne, npts, nv = q.shape
    for _ in range(nsweep):
        Fq = level.stage_residual(q, c_mass, src, S).reshape(ne, npts * nv)
        dq = np.zeros_like(Fq)
        for line in lines:
            dq[line] = line_solve(D, Am, Ap, line, Fq[line])
        q = q + alpha_r * dq.reshape(q.shape)
    return q
