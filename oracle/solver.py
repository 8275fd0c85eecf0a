"""Element-Jacobi smoother, P-level transfers, the FAS V-cycle, pseudo-transient
continuation and the ESDIRK driver (Secs. 2.4 and 3).

Readings, where the paper is silent:
* ||F|| is the Euclidean norm over every solution point and variable of the fine level.
* Pseudo time: dtau_0 = dtau_init at the start of every stage solve; afterwards the SER
  law of eq. (31), dtau_m = min(dtau_{m-1} (r_{m-1}/r_m)^1.5, dtau_max) (optionally never
  below dtau_init: ser_floor, a reading, as eq. (31) states no lower bound), with one global
  dtau shared by all levels. (The CFL form of eqs. (31)-(33) scales the same law by the
  mesh's dtau_min.)
* The smoother D is rebuilt on every level at V-cycles m = 0, k, 2k, ... (k = 10, Sec. 4.1);
  once a rebuild has used dtau = dtau_max no further rebuilds happen (Sec. 4.3). The
  fine-level D is built from q^m, a coarse-level D from that level's restricted state
  q^b inside the same V-cycle.
* A stage solve stops when r_m / r_0 <= tol, r_m = ||F(q^m)|| at the start of V-cycle m.
* q-independent source terms cancel in F_l(q) - S_l on coarse levels (eqs. (40), (43)),
  so only the finest level carries the ESDIRK source.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

from . import gas as G
from .basis import interpolation_1d, projection_1d
from .fr import FRLevel
from .fr3 import FRLevel3
from .geometry import element_dx
from .geometry3d import element_dx3
from .lines import line_blocks, line_sweeps
from .jacobian import element_blocks


# ---- ESDIRK tableaux (eq. (24)); stiffly accurate, first stage explicit -----------
def esdirk_tableau(name: str) -> np.ndarray:
    """Butcher matrix A (s x s); b is the last row and omega = A[1, 1].

    ESDIRK2: the three-stage, L-stable, stiffly accurate scheme with
    gamma = 1 - sqrt(2)/2, c = (0, 2 gamma, 1) (Kennedy & Carpenter, as cited in Sec. 2.4).
    ESDIRK3: the four-stage ESDIRK3(2)4L[2]SA scheme of Kennedy & Carpenter (the
    implicit part of ARK3(2)4L[2]SA), the third-order scheme the paper cites.
    ESDIRK4: the six-stage ESDIRK4(3)6L[2]SA scheme of Kennedy & Carpenter (the implicit part
    of ARK4(3)6L[2]SA), gamma = 1/4, c = (0, 1/2, 83/250, 31/50, 17/20, 1), the fourth-order
    scheme of Sec. 2.4.
    """
    if name == "esdirk2":
        g = 1.0 - math.sqrt(2.0) / 2.0
        b1 = math.sqrt(2.0) / 4.0
        return np.array([[0.0, 0.0, 0.0], [g, g, 0.0], [b1, b1, g]])
    if name == "esdirk3":
        g = 1767732205903.0 / 4055673282236.0
        a31 = 2746238789719.0 / 10658868560708.0
        a32 = -640167445237.0 / 6845629431997.0
        b = [1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0,
             11266239266428.0 / 11593286722821.0, g]
        return np.array([[0.0, 0.0, 0.0, 0.0], [g, g, 0.0, 0.0],
                         [a31, a32, g, 0.0], b])
    if name == "esdirk4":
        g = 0.25
        A = np.zeros((6, 6))
        A[1, :2] = [g, g]
        A[2, :3] = [8611 / 62500, -1743 / 31250, g]
        A[3, :4] = [5012029 / 34652500, -654441 / 2922500, 174375 / 388108, g]
        A[4, :5] = [15267082809 / 155376265600, -71443401 / 120774400, 730878875 / 902184768,
                    2285395 / 8070912, g]
        A[5, :] = [82889 / 524892, 0.0, 15625 / 83664, 69875 / 102672, -2260 / 8211, g]
        return A
    raise ValueError(name)


# ---- transfers (Sec. 3, eqs. (39), (42) restriction; (44), (45) prolongation) --------
def _tensor_apply(A1, x, n_in: int, dim=None):
    """Apply the 1-D matrix A1 along every reference direction of point values x [Ne, n_in^d, Nv]
    (d = 2 or 3, points ordered with the first direction fastest; d from the point count unless
    given, which it must be for n_in = 1)."""
    ne, npts, nv = x.shape
    d = dim if dim is not None else (2 if npts == n_in ** 2 else 3)
    n_out = A1.shape[0]
    if d == 2:
        y = np.einsum("bj,ai,ejiv->ebav", A1, A1, x.reshape(ne, n_in, n_in, nv))
        return y.reshape(ne, n_out ** 2, nv)
    y = np.einsum("ck,bj,ai,ekjiv->ecbav", A1, A1, A1, x.reshape(ne, n_in, n_in, n_in, nv))
    return y.reshape(ne, n_out ** 3, nv)


def restrict(x, Pf: int, Pc: int, dim=None):
    """Tensor-product L2 projection of a [Ne, (Pf+1)^d, Nv] field onto degree Pc."""
    return _tensor_apply(projection_1d(Pf, Pc), x, Pf + 1, dim)


def prolong(x, Pc: int, Pf: int, dim=None):
    """Tensor-product interpolation of a degree-Pc field at the degree-Pf points."""
    return _tensor_apply(interpolation_1d(Pc, Pf), x, Pc + 1, dim)


@dataclass
class PMGOptions:
    p_levels: tuple = (2, 1, 0)          # P{P0-P1-...}
    n_smooth: tuple = (5, 10, 20)        # I{n0-n1-...}; pre = post, coarsest once
    dtau_init: float = 0.01
    dtau_max: float = 10.0
    ser_exp: float = 1.5
    # a lower bound of the SER law at its V-cycle-0 value (the paper states none; a reading)
    ser_floor: bool = False
    refresh_every: int = 10
    freeze_at_max: bool = True
    tol: float = 1e-8
    max_vcycles: int = 200
    alpha_r: float = 1.0
    # CFL form of the pseudo-time step (eqs. (31)-(33)): dtau = CFL dtau_min, CFL from cfl_init
    # to cfl_max by the same SER law (Sec. 4.2 uses 1e2 -> 1e5)
    use_cfl: bool = False
    cfl_init: float = 1e2
    cfl_max: float = 1e5
    # per level: None (element Jacobi) or a [n_lines, K] array of element lines on which that
    # level smooths by element-line Jacobi (``oracle.lines``)
    lines: tuple = ()


@dataclass
class StageStats:
    n_vcycles: int = 0
    r0: float = 0.0
    r_final: float = 0.0
    history: list = field(default_factory=list)
    dtau_history: list = field(default_factory=list)
    refreshes: list = field(default_factory=list)
    converged: bool = False
    dtau_scale: tuple = ()


class PMGSolver:
    """The P-multigrid stage solver on one mesh."""

    def __init__(self, mesh, gas: G.Gas, opts: PMGOptions, q_inf=None):
        self.opts = opts
        self.gas = gas
        level_cls = FRLevel if mesh.dim == 2 else FRLevel3
        self.levels = [level_cls(mesh, P, gas, q_inf) for P in opts.p_levels]
        self.D = [None] * len(self.levels)
        self.c_mass = 0.0
        self.src = None
        self.dtau = opts.dtau_init
        self.refresh_now = False
        self.dtau_last_refresh = None

    # ---- level operators ---------------------------------------------------------
    def F(self, l, q, S=None):
        """F_l(q) - S_l on level l (only level 0 carries the ESDIRK source)."""
        return self.levels[l].stage_residual(q, self.c_mass, self.src if l == 0 else None, S)

    def level_lines(self, l):
        lines = self.opts.lines
        return lines[l] if l < len(lines) else None

    def build_D(self, l, q):
        lines = self.level_lines(l)
        if lines is None:
            self.D[l] = element_blocks(self.levels[l], q, self.dtau, self.c_mass)
        else:
            self.D[l] = line_blocks(self.levels[l], q, self.dtau, self.c_mass, lines)

    def smooth(self, l, q, S, nsweep):
        """Element Jacobi, eq. (30): q <- q + alpha_r D^{-1} (F_l(q) - S_l), all elements at once
        (or element-line Jacobi where the level has lines, ``oracle.lines``)."""
        lev = self.levels[l]
        lines = self.level_lines(l)
        if lines is not None:
            return line_sweeps(lev, q, self.D[l], lines, nsweep, self.c_mass,
                               self.src if l == 0 else None, S, self.opts.alpha_r)
        for _ in range(nsweep):
            Fq = self.F(l, q, S).reshape(lev.ne, lev.n, 1)
            dq = np.linalg.solve(self.D[l], Fq)
            q = q + self.opts.alpha_r * dq.reshape(q.shape)
        return q

    # ---- V-cycle (Sec. 3) --------------------------------------------------------
    def vcycle(self, l, q, S):
        o = self.opts
        last = len(self.levels) - 1
        if self.refresh_now and l > 0:
            self.build_D(l, q)
        q = self.smooth(l, q, S, o.n_smooth[l])           # q^a_l
        if l == last:
            return q
        Pf, Pc = o.p_levels[l], o.p_levels[l + 1]
        d = -self.F(l, q, S)                                # d_l = S_l - F_l(q^a), eqs. (38), (41)
        dim = self.levels[0].mesh.dim
        qb = restrict(q, Pf, Pc, dim)                       # q^b_{l+1}, eqs. (39), (42)
        S1 = self.F(l + 1, qb) + restrict(d, Pf, Pc, dim)   # S_{l+1}, eqs. (40), (43)
        qa1 = self.vcycle(l + 1, qb, S1)
        q = q + prolong(qa1 - qb, Pc, Pf, dim)              # q^{c,b}_l, eqs. (44), (45)
        return self.smooth(l, q, S, o.n_smooth[l])          # q^{c,a}_l

    def residual_norm(self, q):
        return float(np.sqrt(np.sum(self.F(0, q) ** 2)))

    def dtau_min(self, q):
        """dtau_min = min(dtau_inv, dtau_vis) of eq. (33) on the finest level at state q, with
        dtau_inv = min over elements and points of (dx/(P+1)) / (c + |v|) and, when mu > 0,
        dtau_vis = min of (dx/(P+1))^2 / (mu/rho)."""
        lev = self.levels[0]
        if not hasattr(self, "_dx"):
            self._dx = element_dx(lev.mesh) if lev.mesh.dim == 2 else element_dx3(lev.mesh)
        h = (self._dx / (lev.P + 1))[:, None]
        speed = G.sound_speed(q, self.gas) + np.sqrt(np.sum(q[..., 1:-1] ** 2, axis=-1))
        dt = np.min(h / speed)
        if self.gas.mu > 0.0:
            dt = min(dt, np.min(h * h * G.density(q, self.gas) / self.gas.mu))
        return float(dt)

    # ---- pseudo-transient stage solve (Sec. 2.4, eqs. (27)-(31)) -----------------------
    def stage_solve(self, q, c_mass=0.0, src=None, max_vcycles=None):
        o = self.opts
        self.c_mass = c_mass
        self.src = src
        st = StageStats()
        nmax = o.max_vcycles if max_vcycles is None else max_vcycles
        self.dtau_last_refresh = None
        r_prev = None
        if o.use_cfl:
            scale = self.dtau_min(q)
            dtau_init, dtau_max = o.cfl_init * scale, o.cfl_max * scale
        else:
            dtau_init, dtau_max = o.dtau_init, o.dtau_max
        st.dtau_scale = (dtau_init, dtau_max)
        for m in range(nmax + 1):
            r = self.residual_norm(q)
            st.history.append(r)
            if m == 0:
                st.r0 = r
                self.dtau = dtau_init
            else:
                self.dtau = min(self.dtau * (r_prev / r) ** o.ser_exp, dtau_max)
                if o.ser_floor:
                    self.dtau = max(self.dtau, dtau_init)
            st.r_final = r
            if r == 0.0 or r / st.r0 <= o.tol:
                st.converged = True
                break
            if m == nmax:
                break
            st.dtau_history.append(self.dtau)
            frozen = (o.freeze_at_max and self.dtau_last_refresh is not None
                      and self.dtau_last_refresh >= dtau_max)
            self.refresh_now = m == 0 or (m % o.refresh_every == 0 and not frozen)
            if self.refresh_now:
                self.build_D(0, q)
                self.dtau_last_refresh = self.dtau
                st.refreshes.append(m)
            q = self.vcycle(0, q, None)
            st.n_vcycles = m + 1
            r_prev = r
        return q, st

    # ---- Newton-Krylov stage solve with the V-cycle as preconditioner ---------------------
    def nk_stage_solve(self, q, c_mass=0.0, src=None, krylov_dim=10, eta=1e-2, max_newton=None,
                       fd_rel=1e-3, pc_rel=1e-3, precondition=True):
        """Pseudo-transient Newton on F(q) = 0 with the whole Jacobian (the linearisation of
        eqs. (27)-(28) without the element-Jacobi splitting of eq. (29)): at step m,

            (Gamma(q_m)/dtau_m - dF/dq) delta = F(q_m),   q_{m+1} = q_m + delta,

        solved by one cycle of flexible GMRES from delta = 0 with at most krylov_dim directions,
        stopped once the least-squares residual is <= eta ||F(q_m)||. Products with dF/dq are
        forward differences (F(q_m + h z) - F(q_m))/h with h ||z|| = fd_rel sqrt(N) (N entries of
        the state): fd_rel is the RMS size of the perturbation per entry, of the order of
        sqrt(machine epsilon) times the absolute state (1e-3 for pressures near 6e4 at Ma 0.005). The right preconditioner is one FAS V-cycle of Sec. 3 started at q_m on
        F(q) - S_0 = 0 with S_0 = F(q_m) - e v, whose first sweep moves q_m by e D^{-1} v:
        M^{-1} v = (V(q_m) - q_m)/e with e = pc_rel sqrt(N) (||v|| = 1). Orthogonalisation: classical
        Gram-Schmidt applied twice, then the norm of the orthogonalised vector itself.
        dtau follows the SER law of eq. (31) and the blocks are rebuilt
        as in stage_solve (the coarse ones in the first preconditioner V-cycle of a refresh step).
        The history holds ||F|| per Newton step; st.krylov counts the directions taken."""
        o = self.opts
        self.c_mass = c_mass
        self.src = src
        st = StageStats()
        st.krylov = 0
        nmax = o.max_vcycles if max_newton is None else max_newton
        self.dtau_last_refresh = None
        r_prev = None
        if o.use_cfl:
            scale = self.dtau_min(q)
            dtau_init, dtau_max = o.cfl_init * scale, o.cfl_max * scale
        else:
            dtau_init, dtau_max = o.dtau_init, o.dtau_max
        sqn = math.sqrt(q.size)
        for m in range(nmax + 1):
            F0 = self.F(0, q)
            r = float(np.sqrt(np.sum(F0 ** 2)))
            st.history.append(r)
            if m == 0:
                st.r0 = r
                self.dtau = dtau_init
            else:
                self.dtau = min(self.dtau * (r_prev / r) ** o.ser_exp, dtau_max)
                if o.ser_floor:
                    self.dtau = max(self.dtau, dtau_init)
            st.r_final = r
            if r == 0.0 or r / st.r0 <= o.tol:
                st.converged = True
                break
            if m == nmax:
                break
            st.dtau_history.append(self.dtau)
            frozen = (o.freeze_at_max and self.dtau_last_refresh is not None
                      and self.dtau_last_refresh >= dtau_max)
            refresh_coarse = False
            if m == 0 or (m % o.refresh_every == 0 and not frozen):
                self.build_D(0, q)
                self.dtau_last_refresh = self.dtau
                st.refreshes.append(m)
                refresh_coarse = True
            gam = G.preconditioner(q, self.gas)
            k = krylov_dim
            V = [F0 / r]
            Z = []
            H = np.zeros((k + 1, k))
            cs, sn = np.zeros(k), np.zeros(k)
            g = np.zeros(k + 1)
            g[0] = r
            jj = 0
            for j in range(k):
                v = V[j]
                if precondition:
                    e = pc_rel * sqn                        # ||v|| = 1 by construction
                    self.refresh_now = refresh_coarse
                    refresh_coarse = False
                    z = (self.vcycle(0, q.copy(), F0 - e * v) - q) / e
                    self.refresh_now = False
                else:
                    z = v
                Z.append(z)
                h = fd_rel * sqn / float(np.sqrt(np.sum(z ** 2)))
                w = np.einsum("...ij,...j->...i", gam, z) / self.dtau - (self.F(0, q + h * z) - F0) / h
                c = np.array([float(np.sum(Vi * w)) for Vi in V])       # classical Gram-Schmidt
                w = w - sum(ci * Vi for ci, Vi in zip(c, V))
                H[:j + 1, j] += c
                c = np.array([float(np.sum(Vi * w)) for Vi in V])       # applied again
                w = w - sum(ci * Vi for ci, Vi in zip(c, V))
                H[:j + 1, j] += c
                H[j + 1, j] = math.sqrt(float(np.sum(w * w)))
                for i in range(j):                          # earlier rotations, then a new one
                    a, b = H[i, j], H[i + 1, j]
                    H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * b, -sn[i] * a + cs[i] * b
                den = math.hypot(H[j, j], H[j + 1, j])
                cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
                hn = H[j + 1, j]
                H[j, j], H[j + 1, j] = den, 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                jj = j + 1
                if abs(g[j + 1]) <= eta * r or hn == 0.0:
                    break
                V.append(w / hn)
            y = np.zeros(jj)
            for i in range(jj - 1, -1, -1):
                y[i] = (g[i] - H[i, i + 1:jj] @ y[i + 1:jj]) / H[i, i]
            q = q + sum(yi * zi for yi, zi in zip(y, Z))
            st.krylov += jj
            st.n_vcycles = m + 1
            r_prev = r
        return q, st

    # ---- ESDIRK step (eqs. (24)-(26)) -----------------------------------------------
    def esdirk_step(self, q_n, dt, tableau: np.ndarray, stage_guess: str = "previous"):
        """One step of eq. (24), every implicit stage i solved by stage_solve from an initial guess
        the paper does not state:
        * "previous" (default): the previous stage value q^{i-1};
        * "predictor": the stage equation evaluated with R(q^i) replaced by the previous stage's
          residual, q_c = q_c^n + dt sum_{j<i} a_ij R_j + dt omega R_{i-1}, converted to primitive
          variables. Once q^n is a solved time level, a stage started from the previous stage
          value begins so close to its solution that the first V-cycle's element-Jacobi sweeps
          raise the continuity and energy residuals by orders of magnitude against that tiny r_0,
          and the SER law then collapses dtau; from the predictor the relative residual falls
          steadily (Sec. 4.1 setting: tol 1e-4 within about a dozen V-cycles). From an unsolved
          initial condition R(q^n) carries the truncation error and the predictor is far off, so
          the first step of a run uses "previous"."""
        lev0 = self.levels[0]
        A = tableau
        s = A.shape[0]
        omega = A[1, 1]
        qc_n = G.conservative(q_n, self.gas)
        Rs = [lev0.residual(q_n)]
        q = q_n
        stats = []
        for i in range(1, s):
            acc = qc_n.copy()
            for j in range(i):
                acc = acc + dt * A[i, j] * Rs[j]
            src = acc / (omega * dt)
            if stage_guess == "predictor":
                q = G.primitive(acc + dt * omega * Rs[i - 1], self.gas)
            elif stage_guess != "previous":
                raise ValueError(stage_guess)
            q, st = self.stage_solve(q, c_mass=1.0 / (omega * dt), src=src)
            stats.append(st)
            Rs.append(lev0.residual(q))
        return q, stats
