"""Oracle patches: an element and its face neighbours as a mesh of their own. The element block
of eq. (30) holds the neighbours' states fixed, so the patch gives the same block as the whole
mesh; tests use it to check sampled elements of the full-size meshes."""
from __future__ import annotations

import numpy as np

import workloads as W


def patch_mesh(mesh, e):
    """The element e and its face neighbours (e first) and their global indices; faces that lead
    out of the patch become far-field faces (they change only the neighbours' residuals)."""
    elems = [e]
    for nb in mesh.face_nbr[e]:
        if nb >= 0 and int(nb) not in elems:
            elems.append(int(nb))
    local = {g: k for k, g in enumerate(elems)}
    nf = mesh.face_nbr.shape[1]
    fn = np.full((len(elems), nf), W.BC_FAR_FIELD, np.int32)
    fnf = np.zeros((len(elems), nf), np.int32)
    fo = np.zeros((len(elems), nf), np.int32)
    for k, g in enumerate(elems):
        for f in range(nf):
            nb = int(mesh.face_nbr[g, f])
            if nb < 0:
                fn[k, f] = nb
            elif nb in local:
                fn[k, f] = local[nb]
                fnf[k, f] = mesh.face_nbr_face[g, f]
                fo[k, f] = mesh.face_orient[g, f]
    return W.Mesh(mesh.dim, mesh.geom_order, mesh.nodes[elems].copy(), fn, fnf, fo), elems


def patch_block(mesh, gas, P, q, e, dtau, c_mass, q_inf):
    """The oracle's block D_e (eqs. (28), (30)) of element e of the whole mesh, from its patch."""
    from oracle.fr import FRLevel
    from oracle.fr3 import FRLevel3
    from oracle.jacobian import element_blocks
    pm, elems = patch_mesh(mesh, e)
    lev = (FRLevel if mesh.dim == 2 else FRLevel3)(pm, P, gas, q_inf=q_inf)
    return element_blocks(lev, q[elems], dtau, c_mass)[0]
