"""Seeded synthetic workloads shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the solver. It produces

* meshes: element geometry nodes, face connectivity and boundary tags;
* the closed-form isentropic vortex of the accuracy study (Sec. 4.1, eq. (46)),
  as a pointwise function of physical coordinates and time.

Both the oracle and the GPU path evaluate the vortex at their own solution
points, which each side computes itself.

Conventions
-----------
* Geometry nodes of an element are in tensor order, xi fastest:
  node ``a + (g+1)*b`` sits at reference coordinates
  ``(-1 + 2a/g, -1 + 2b/g)`` for geometry order ``g`` (1 = bilinear, 2 = 9-node).
* Faces of a quad: 0 = (xi=-1), 1 = (xi=+1), 2 = (eta=-1), 3 = (eta=+1).
* ``face_nbr[e, f] >= 0`` is the neighbour element; a negative value is a boundary
  tag (``BC_SLIP_WALL``, ``BC_FAR_FIELD``).
* ``face_nbr_face[e, f]`` is the neighbour's face index and ``face_orient[e, f]``
  is 0 when flux point k meets the neighbour's flux point k, 1 when it meets
  point ``P-k`` (reversed edge direction).
* Hexahedra (``dim == 3``): node ``a + (g+1)*b + (g+1)^2*c`` sits at
  ``(-1 + 2a/g, -1 + 2b/g, -1 + 2c/g)``; faces 0/1 = (xi = -1/+1), 2/3 = (eta = -1/+1),
  4/5 = (zeta = -1/+1). A face's points are indexed (k1, k2) along its two tangential
  reference directions in increasing order ((eta, zeta), (xi, zeta), (xi, eta)).
  ``face_orient`` (0..7) maps (k1, k2) to the neighbour's face point: swap the pair if bit 0
  is set, then reverse the first index (``P - k``) if bit 1 is set and the second if bit 2 is.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BC_SLIP_WALL = -1
BC_FAR_FIELD = -2
BC_NOSLIP_WALL = -3

JITTER_SEED = 20190811


@dataclass
class Mesh:
    dim: int
    geom_order: int
    nodes: np.ndarray          # [Ne, (g+1)^d, d] float64
    face_nbr: np.ndarray       # [Ne, 2d] int32
    face_nbr_face: np.ndarray  # [Ne, 2d] int32
    face_orient: np.ndarray    # [Ne, 2d] int32
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(self.nodes.shape[0])


def periodic_quad_mesh(n: int, length: float = 10.0, jitter: float = 0.0,
                       seed: int = JITTER_SEED, origin: float | None = None) -> Mesh:
    """Bilinear quads on the periodic square ``[origin, origin+length]^2``, n x n cells.

    With ``jitter > 0`` every vertex is moved by independent ``U(-jitter*h, jitter*h)``
    offsets in x and in y (``h = length/n``), drawn from ``numpy.random.default_rng(seed)``:
    first the n x n array of x offsets, then the n x n array of y offsets, indexed
    ``[i, j]`` with i the x index. Offsets belong to a periodic vertex class
    (index mod n), so opposite sides of the box stay matched.
    Elements are numbered ``e = i + n*j`` (x index fastest).
    """
    return periodic_rect_mesh(n, n, length, length, jitter, seed, origin, origin)


def periodic_rect_mesh(nx: int, ny: int, lx: float = 10.0, ly: float = 10.0, jitter: float = 0.0,
                       seed: int = JITTER_SEED, ox: float | None = None, oy: float | None = None) -> Mesh:
    """Bilinear quads on a periodic nx x ny box (see ``periodic_quad_mesh`` for the jitter recipe,
    here with offsets of shape (nx, ny) scaled by each direction's cell size)."""
    ox = -0.5 * lx if ox is None else ox
    oy = -0.5 * ly if oy is None else oy
    hx, hy = lx / nx, ly / ny
    dx = np.zeros((nx, ny))
    dy = np.zeros((nx, ny))
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        dx = rng.uniform(-jitter * hx, jitter * hx, size=(nx, ny))
        dy = rng.uniform(-jitter * hy, jitter * hy, size=(nx, ny))
    ne = nx * ny
    nodes = np.zeros((ne, 4, 2))
    nbr = np.zeros((ne, 4), np.int32)
    nbf = np.zeros((ne, 4), np.int32)
    ori = np.zeros((ne, 4), np.int32)
    for j in range(ny):
        for i in range(nx):
            e = i + nx * j
            for b in range(2):
                for a in range(2):
                    vi, vj = i + a, j + b
                    nodes[e, a + 2 * b, 0] = ox + vi * hx + dx[vi % nx, vj % ny]
                    nodes[e, a + 2 * b, 1] = oy + vj * hy + dy[vi % nx, vj % ny]
            nbr[e, 0] = (i - 1) % nx + nx * j
            nbr[e, 1] = (i + 1) % nx + nx * j
            nbr[e, 2] = i + nx * ((j - 1) % ny)
            nbr[e, 3] = i + nx * ((j + 1) % ny)
            nbf[e] = (1, 0, 3, 2)
    return Mesh(2, 1, nodes, nbr, nbf, ori, name=f"periodic{nx}x{ny}",
                info={"length": (lx, ly), "origin": (ox, oy), "jitter": jitter,
                      "seed": seed if jitter > 0 else None, "periodic": True})


def channel_mesh(nx: int, ny: int, lx: float = 10.0, ly: float = 2.0, jitter: float = 0.0,
                 seed: int = JITTER_SEED, wall: int = BC_NOSLIP_WALL) -> Mesh:
    """Bilinear quads on [0, lx] x [0, ly], periodic in x, with a wall of type ``wall`` at
    y = 0 and y = ly (interior vertices jittered as in ``periodic_rect_mesh``; wall vertices keep
    their y)."""
    m = periodic_rect_mesh(nx, ny, lx, ly, jitter, seed, ox=0.0, oy=0.0)
    nodes = m.nodes.copy()
    nbr = m.face_nbr.copy()
    for j in range(ny):
        for i in range(nx):
            e = i + nx * j
            for b in range(2):
                if j + b in (0, ny):          # vertices on a wall stay on it
                    for a in range(2):
                        nodes[e, a + 2 * b, 1] = 0.0 if j + b == 0 else ly
            if j == 0:
                nbr[e, 2] = wall
            if j == ny - 1:
                nbr[e, 3] = wall
    return Mesh(2, 1, nodes, nbr, m.face_nbr_face, m.face_orient, name=f"channel{nx}x{ny}",
                info={"length": (lx, ly), "jitter": jitter, "seed": seed if jitter > 0 else None, "wall": wall})


@dataclass
class VortexSpec:
    """Isentropic vortex of Sec. 4.1 (eq. (46)).

    ``ma_ref`` names the speed the free-stream Mach number is referred to, which the
    paper does not fix: ``"speed"`` uses |V_inf| (= sqrt(2) for u=v=1), ``"u"`` uses u_inf.
    Gas constant R = 1 (so T = p/rho); this is the value for which the printed
    temperature perturbation is the exact isentropic balance.
    """
    gamma: float = 1.4
    rgas: float = 1.0
    rho_inf: float = 1.0
    u_inf: tuple = (1.0, 1.0)
    ma_inf: float = 0.005
    ma_ref: str = "speed"
    alpha: float = 5.0
    phi: float = 0.5
    center: tuple = (0.0, 0.0)
    length: float = 10.0       # periodic box length, used to pick the nearest image

    @property
    def c_inf(self) -> float:
        ref = math.hypot(*self.u_inf) if self.ma_ref == "speed" else self.u_inf[0]
        return ref / self.ma_inf

    @property
    def t_inf(self) -> float:
        return self.c_inf ** 2 / (self.gamma * self.rgas)

    @property
    def p_inf(self) -> float:
        return self.rho_inf * self.rgas * self.t_inf

    def freestream(self) -> np.ndarray:
        """Primitive free-stream state (p, u, v, T)."""
        return np.array([self.p_inf, self.u_inf[0], self.u_inf[1], self.t_inf])

    def state(self, x: np.ndarray, y: np.ndarray, t: float = 0.0) -> np.ndarray:
        """Primitive state (p, u, v, T) of the vortex advected to time t, shape x.shape + (4,)."""
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        L = self.length
        xr = x - self.center[0] - self.u_inf[0] * t
        yr = y - self.center[1] - self.u_inf[1] * t
        xr = xr - L * np.round(xr / L)
        yr = yr - L * np.round(yr / L)
        r2 = xr * xr + yr * yr
        g = self.gamma
        amp = self.alpha / (2.0 * math.pi)
        ex = np.exp(self.phi * (1.0 - r2))
        du = -amp * yr * ex
        dv = amp * xr * ex
        dT = -(self.alpha ** 2) * (g - 1.0) / (16.0 * self.phi * g * math.pi ** 2) * ex * ex
        T = self.t_inf + dT
        rho = self.rho_inf * (T / self.t_inf) ** (1.0 / (g - 1.0))
        p = rho * self.rgas * T
        return np.stack([p, self.u_inf[0] + du, self.u_inf[1] + dv, T], axis=-1)


def vortex_config1() -> tuple[Mesh, VortexSpec]:
    """8x8 uniform periodic quads on [-5,5]^2 (the small parity case)."""
    return periodic_quad_mesh(8, 10.0), VortexSpec(length=10.0)


def vortex_config2() -> tuple[Mesh, VortexSpec]:
    """64x64 periodic quads on [-5,5]^2, vertices jittered by +-10% of the cell size."""
    return periodic_quad_mesh(64, 10.0, jitter=0.1, seed=JITTER_SEED), VortexSpec(length=10.0)


# ---- airfoil O-mesh (synthetic stand-in for the NACA0012 meshes of Sec. 4.2) --------------
def naca4_symmetric_half_thickness(x: np.ndarray, t: float = 0.12) -> np.ndarray:
    """Half thickness of the symmetric 4-digit profile with the closed-trailing-edge coefficient."""
    x = np.clip(np.asarray(x, float), 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2 + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def airfoil_o_mesh(n_wrap: int = 128, n_radial: int = 64, ratio: float = 1.1, r_far: float = 20.0,
                   thickness: float = 0.12, annulus: bool = False, wall: int = BC_SLIP_WALL) -> Mesh:
    """9-node quadratic O-mesh around a closed-TE symmetric 4-digit profile (chord 1).

    Wrap direction (xi): surface points at angle theta = 2 pi s / n_wrap (s in half steps for the
    mid-edge nodes), x = (1 + cos theta)/2 (cosine clustering), y = -y_t(x) for sin theta > 0 and
    +y_t(x) otherwise, i.e. the surface is walked clockwise so that (xi, eta) is right-handed.
    Radial direction (eta): straight lines from each surface point to the far-field circle point
    (0.5 + r_far cos theta, -r_far sin theta), node fractions (ratio^k - 1)/(ratio^n - 1) with k in
    half steps (first cell height ~ r_far * (ratio - 1)/(ratio^n - 1)).
    Faces: xi faces wrap periodically; eta = -1 of the first layer is a wall of type ``wall`` (slip
    by default, ``BC_NOSLIP_WALL`` for viscous flow), eta = +1 of the last layer far field. With annulus=True the profile is replaced by the unit circle and the
    inner boundary is also far field (a curved mesh for free-stream tests).
    Element e = i + n_wrap * j.
    """
    nw, nr = n_wrap, n_radial
    s_half = np.arange(2 * nw + 1) / 2.0                       # wrap positions in half cells
    theta = 2.0 * np.pi * s_half / nw
    if annulus:
        xs, ys = np.cos(theta), -np.sin(theta)
        cx = 0.0
    else:
        xs = 0.5 * (1.0 + np.cos(theta))
        yt = naca4_symmetric_half_thickness(xs, thickness)
        ys = np.where(np.sin(theta) > 0.0, -yt, yt)
        ys[np.abs(np.sin(theta)) < 1e-15] = 0.0
        cx = 0.5
    xf, yf = cx + r_far * np.cos(theta), -r_far * np.sin(theta)
    k_half = np.arange(2 * nr + 1) / 2.0
    frac = (ratio ** k_half - 1.0) / (ratio ** nr - 1.0)
    X = xs[:, None] + frac[None, :] * (xf - xs)[:, None]        # [2nw+1, 2nr+1]
    Y = ys[:, None] + frac[None, :] * (yf - ys)[:, None]
    ne = nw * nr
    nodes = np.zeros((ne, 9, 2))
    nbr = np.zeros((ne, 4), np.int32)
    nbf = np.zeros((ne, 4), np.int32)
    for j in range(nr):
        for i in range(nw):
            e = i + nw * j
            for b in range(3):
                for a in range(3):
                    nodes[e, a + 3 * b] = (X[2 * i + a, 2 * j + b], Y[2 * i + a, 2 * j + b])
            nbr[e, 0] = (i - 1) % nw + nw * j
            nbr[e, 1] = (i + 1) % nw + nw * j
            nbr[e, 2] = (i + nw * (j - 1)) if j > 0 else (BC_FAR_FIELD if annulus else wall)
            nbr[e, 3] = (i + nw * (j + 1)) if j < nr - 1 else BC_FAR_FIELD
            nbf[e] = (1, 0, 3, 2)
    name = f"{'annulus' if annulus else 'airfoil'}_o{nw}x{nr}"
    return Mesh(2, 2, nodes, nbr, nbf, np.zeros_like(nbr), name=name,
                info={"ratio": ratio, "r_far": r_far, "thickness": thickness, "annulus": annulus})


@dataclass
class FreeStreamSpec:
    """Uniform low-Mach free stream at incidence (Sec. 4.2): rho = 1, |V| = 1, c = |V|/Ma, R = 1."""
    gamma: float = 1.4
    rgas: float = 1.0
    ma_inf: float = 0.001
    alpha_deg: float = 2.0

    def freestream(self) -> np.ndarray:
        a = math.radians(self.alpha_deg)
        c = 1.0 / self.ma_inf
        t = c * c / (self.gamma * self.rgas)
        return np.array([self.rgas * t, math.cos(a), math.sin(a), t])


def airfoil_config3(n_wrap: int = 128, n_radial: int = 64) -> tuple[Mesh, FreeStreamSpec]:
    """Inviscid flow at Ma 0.001, 2 degrees incidence around the 12% symmetric profile."""
    return airfoil_o_mesh(n_wrap, n_radial), FreeStreamSpec()


@dataclass
class ViscousCase:
    """One case of the viscous batch: incidence, solution degree and its P-level hierarchy."""
    alpha_deg: float
    P: int
    p_levels: tuple
    spec: FreeStreamSpec
    mu: float
    prandtl: float = 0.72


VISCOUS_SEED = 5000
# P-level hierarchies of the viscous cases: P-jumps of one at P = 4 (with BR2 the P4 -> P2 coarse
# correction diverges on the stretched O-mesh, in the CPU reference as well)
VISCOUS_HIERARCHY = {4: (4, 3, 2, 1), 3: (3, 2, 1), 2: (2, 1, 0)}


def viscous_config4(n_wrap: int = 256, n_radial: int = 96, n_cases: int = 8, reynolds: float = 5000.0,
                    seed: int = VISCOUS_SEED) -> tuple[Mesh, list]:
    """Viscous flow at Re 5000 (mu = rho |V| c / Re with rho = |V| = c = 1), Ma 0.001, around the
    12% profile on the O-mesh refined to n_wrap x n_radial with a no-slip adiabatic wall; n_cases
    independent cases with incidence U[0, 6] degrees and P in {2, 3, 4} drawn from
    default_rng(seed) (incidences first, then degrees)."""
    mesh = airfoil_o_mesh(n_wrap, n_radial, wall=BC_NOSLIP_WALL)
    rng = np.random.default_rng(seed)
    alphas = rng.uniform(0.0, 6.0, n_cases)
    degrees = rng.choice([2, 3, 4], n_cases)
    cases = [ViscousCase(float(a), int(P), VISCOUS_HIERARCHY[int(P)], FreeStreamSpec(alpha_deg=float(a)),
                         mu=1.0 / reynolds) for a, P in zip(alphas, degrees)]
    return mesh, cases


def wall_distance(xy: np.ndarray, thickness: float = 0.12, n_surface: int = 4001) -> np.ndarray:
    """Distance of points xy [..., 2] to the closed-TE symmetric profile (chord 1), by the nearest
    of n_surface cosine-spaced surface points."""
    from scipy.spatial import cKDTree
    x = 0.5 * (1.0 - np.cos(np.linspace(0.0, np.pi, n_surface // 2 + 1)))
    yt = naca4_symmetric_half_thickness(x, thickness)
    surf = np.concatenate([np.stack([x, yt], -1), np.stack([x, -yt], -1)])
    d, _ = cKDTree(surf).query(xy.reshape(-1, 2))
    return d.reshape(xy.shape[:-1])


def viscous_start_state(spec: FreeStreamSpec, xy: np.ndarray, delta: float = 0.05) -> np.ndarray:
    """Initial state of the viscous cases: the free stream with its velocity ramped to zero at the
    wall, u = u_inf tanh(d / delta) (d: wall distance), p and T uniform; it replaces the impulsive
    start of a uniform flow against a no-slip wall."""
    q = np.broadcast_to(spec.freestream(), xy.shape[:-1] + (4,)).copy()
    ramp = np.tanh(wall_distance(xy) / delta)
    q[..., 1] *= ramp
    q[..., 2] *= ramp
    return q


# ---- 3-D: cubed sphere (Sec. 4.2's sphere setting at the sizes of the synthetic config) ------

def face_point_map(orient: int, k1, k2, n1: int):
    """The neighbour's face point (k1', k2') met by point (k1, k2) of a hexahedron face, for the
    ``face_orient`` code documented above (n1 points per direction)."""
    a, b = (k2, k1) if orient & 1 else (k1, k2)
    if orient & 2:
        a = n1 - 1 - a
    if orient & 4:
        b = n1 - 1 - b
    return a, b


_HEX_FACE_CENTER = (12, 14, 10, 16, 4, 22)      # node at the middle of each face (27-node hex)


def _hex_face_nodes(f: int) -> np.ndarray:
    """27-node indices of face f as a 3x3 array [k1][k2] in the face's tangential order."""
    fixed = (0, 2, 0, 2, 0, 2)[f]
    out = np.zeros((3, 3), int)
    for k1 in range(3):
        for k2 in range(3):
            if f < 2:
                a, b, c = fixed, k1, k2
            elif f < 4:
                a, b, c = k1, fixed, k2
            else:
                a, b, c = k1, k2, fixed
            out[k1, k2] = a + 3 * b + 9 * c
    return out


def connect_hex_mesh(nodes: np.ndarray, boundary_tag) -> tuple:
    """Face neighbours, neighbour faces and orientation codes of a conforming 27-node hex mesh, by
    matching face-centre nodes and then the 3x3 face node grids; ``boundary_tag(e, f)`` gives the
    tag of faces without a partner."""
    ne = nodes.shape[0]
    scale = float(np.max(np.abs(nodes)))
    centers = nodes[:, list(_HEX_FACE_CENTER)].reshape(ne * 6, 3)
    keys = np.round(centers / scale * 1e9).astype(np.int64)
    _, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if np.any(counts > 2):
        raise ValueError("more than two faces share a centre")
    order = np.argsort(inv, kind="stable")
    nbr = np.zeros(ne * 6, np.int32)
    nbf = np.zeros(ne * 6, np.int32)
    ori = np.zeros(ne * 6, np.int32)
    grids = np.stack([_hex_face_nodes(f) for f in range(6)])          # [6, 3, 3]
    perms = np.zeros((8, 3, 3, 2), int)
    for o in range(8):
        for k1 in range(3):
            for k2 in range(3):
                perms[o, k1, k2] = face_point_map(o, k1, k2, 3)
    sorted_inv = inv[order]
    starts = np.r_[0, np.nonzero(np.diff(sorted_inv))[0] + 1]
    ends = np.r_[starts[1:], len(order)]
    pairs = [(order[a_], order[a_ + 1]) for a_, b_ in zip(starts, ends) if b_ - a_ == 2]
    singles = [order[a_] for a_, b_ in zip(starts, ends) if b_ - a_ == 1]
    for x in singles:
        nbr[x] = boundary_tag(x // 6, x % 6)
    if pairs:
        pa = np.array(pairs)
        for side in (0, 1):
            me, th = pa[:, side], pa[:, 1 - side]
            e, f, g, h = me // 6, me % 6, th // 6, th % 6
            mine = nodes[e[:, None, None], grids[f]]                    # [m, 3, 3, 3]
            theirs = nodes[g[:, None, None], grids[h]]
            best = np.full(len(me), -1)
            for o in range(7, -1, -1):
                t = theirs[:, perms[o, :, :, 0], perms[o, :, :, 1]]
                ok = np.all(np.abs(mine - t) <= 1e-9 * scale, axis=(1, 2, 3))
                best = np.where(ok, o, best)
            if np.any(best < 0):
                raise ValueError("face node grids do not match")
            nbr[me], nbf[me], ori[me] = g, h, best
    return nbr.reshape(ne, 6), nbf.reshape(ne, 6), ori.reshape(ne, 6)


# cube-face frames (t1, t2, n) of the six patches, right-handed (t1 x t2 = n)
_CUBE_FRAMES = (
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, 0, 1), (0, 1, 0), (-1, 0, 0)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((1, 0, 0), (0, 0, 1), (0, -1, 0)),
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((0, 1, 0), (1, 0, 0), (0, 0, -1)),
)


def cubed_sphere_mesh(n: int = 16, n_shells: int = 24, ratio: float = 1.1, r_far: float = 20.0,
                      r_in: float = 1.0, inner: int = BC_SLIP_WALL) -> Mesh:
    """Equiangular cubed sphere of 27-node hexahedra between radii r_in and r_far.

    Six patches (cube faces) of n x n cells: on a patch with frame (t1, t2, n) the direction of the
    angles (a, b) in [-pi/4, pi/4]^2 is (n + tan a t1 + tan b t2) normalised (xi along a, eta along
    b). Radial shells (zeta, outwards): node fractions (ratio^k - 1)/(ratio^n_shells - 1) with k in
    half steps (first shell height (r_far - r_in)(ratio - 1)/(ratio^n_shells - 1)). Nodes lie on the
    exact map; zeta = -1 of the first shell is the sphere (tag ``inner``), zeta = +1 of the last
    shell far field. Element e = i + n (j + n (patch + 6 k)) for cell (i, j) of a patch and shell k.
    """
    ang = -0.25 * np.pi + 0.5 * np.pi * np.arange(2 * n + 1) / (2 * n)
    k_half = np.arange(2 * n_shells + 1) / 2.0
    rad = r_in + (r_far - r_in) * (ratio ** k_half - 1.0) / (ratio ** n_shells - 1.0)
    ne = 6 * n * n * n_shells
    nodes = np.zeros((n_shells, 6, n, n, 3, 3, 3, 3))              # [k, p, j, i, c, b, a, xyz]
    ta = np.tan(ang)
    ia = 2 * np.arange(n)[:, None] + np.arange(3)[None, :]         # [cell, node] half-step index
    for p, (t1, t2, nn) in enumerate(_CUBE_FRAMES):
        t1, t2, nn = np.array(t1, float), np.array(t2, float), np.array(nn, float)
        d = (nn[None, None, None, None, :] + ta[ia][None, None, :, :, None] * t1
             + ta[ia][:, :, None, None, None] * t2)                  # [j, b, i, a, xyz]
        d = d / np.linalg.norm(d, axis=-1, keepdims=True)
        r = rad[2 * np.arange(n_shells)[:, None] + np.arange(3)[None, :]]   # [k, c]
        # -> [k, j, i, c, b, a, xyz]
        x = r[:, None, None, :, None, None, None] * np.transpose(d, (0, 2, 1, 3, 4))[None, :, :, None, :, :, :]
        nodes[:, p] = x
    nodes = nodes.reshape(ne, 27, 3)
    cells = n * n * 6

    def tag(e, f):
        if f == 4 and e < cells:
            return inner
        if f == 5 and e >= cells * (n_shells - 1):
            return BC_FAR_FIELD
        raise ValueError(f"unmatched interior face ({e},{f})")

    nbr, nbf, ori = connect_hex_mesh(nodes, tag)
    return Mesh(3, 2, nodes, nbr, nbf, ori, name=f"cubed_sphere_{n}x{n}x{n_shells}",
                info={"ratio": ratio, "r_far": r_far, "r_in": r_in})


@dataclass
class FreeStream3Spec:
    """Uniform low-Mach free stream along +x (Sec. 4.2 sphere setting): rho = 1, |V| = 1,
    c = |V|/Ma, R = 1; primitive variables (p, u, v, w, T)."""
    gamma: float = 1.4
    rgas: float = 1.0
    ma_inf: float = 0.001

    def freestream(self) -> np.ndarray:
        c = 1.0 / self.ma_inf
        t = c * c / (self.gamma * self.rgas)
        return np.array([self.rgas * t, 1.0, 0.0, 0.0, t])


def sphere_config5(n: int = 16, n_shells: int = 24) -> tuple[Mesh, FreeStream3Spec]:
    """Inviscid flow at Ma 0.001 past the unit sphere on the 6 x 16 x 16 x 24 cubed sphere."""
    return cubed_sphere_mesh(n, n_shells), FreeStream3Spec()

