"""Thin Python binding of the pmgfr C ABI: the same entry points, taking torch tensors for device
memory and the current torch stream. It only marshals arguments; every computation runs in the
HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Level:
    """One P-level of a quadrilateral or hexahedral mesh (a ``pmg_level`` handle)."""

    def __init__(self, mesh, P: int, *, gamma: float = 1.4, rgas: float = 1.0, eps_mode: int = 0,
                 ma_inf: float = 0.0, kappa: float = 1.0, q_inf=None, q_ref=None, device: int = 0,
                 mu: float = 0.0, prandtl: float = 0.72, br2_penalty: float = 4.0):
        lib = A.lib()
        nodes = np.ascontiguousarray(mesh.nodes, dtype=np.float64)
        nbr = np.ascontiguousarray(mesh.face_nbr, dtype=np.int32)
        nbf = np.ascontiguousarray(mesh.face_nbr_face, dtype=np.int32)
        ori = np.ascontiguousarray(mesh.face_orient, dtype=np.int32)
        d = A.LevelDesc()
        d.dim, d.P, d.geom_order, d.n_elements = mesh.dim, P, mesh.geom_order, mesh.n_elements
        d.nodes = nodes.ctypes.data_as(C.POINTER(C.c_double))
        d.face_nbr = nbr.ctypes.data_as(C.POINTER(C.c_int32))
        d.face_nbr_face = nbf.ctypes.data_as(C.POINTER(C.c_int32))
        d.face_orient = ori.ctypes.data_as(C.POINTER(C.c_int32))
        d.gamma, d.rgas, d.eps_mode, d.ma_inf, d.kappa = gamma, rgas, eps_mode, ma_inf, kappa
        qi = np.zeros(5)
        if q_inf is not None:
            qi[:len(q_inf)] = q_inf
        d.q_inf = (C.c_double * 5)(*qi)
        qr = np.zeros(5)
        if q_ref is not None:
            qr[:len(q_ref)] = q_ref
        d.q_ref = (C.c_double * 5)(*qr)
        d.device = device
        d.mu, d.prandtl, d.br2_penalty = mu, prandtl, br2_penalty
        h = A.pmg_level()
        A.check(lib.pmg_level_create(C.byref(d), C.byref(h)), "pmg_level_create")
        self.handle = h
        info = (C.c_int32 * 8)()
        A.check(lib.pmg_level_info(h, info), "pmg_level_info")
        self.dim, self.P, self.np, self.nv, self.n, self.ne, self.device, self.geom_order = list(info)
        self.shape = (self.nv, self.np, self.ne)
        self.q_ref = qr[:self.nv].copy()
        self.torch_device = torch.device("cuda", self.device)

    def points(self) -> np.ndarray:
        """Solution-point coordinates [dim, Np, Ne]."""
        out = np.empty((self.dim, self.np, self.ne))
        A.check(A.lib().pmg_level_points(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))),
                "pmg_level_points")
        return out

    def dx(self) -> np.ndarray:
        """Element length scale of eqs. (32)-(33), [Ne]."""
        out = np.empty(self.ne)
        A.check(A.lib().pmg_level_dx(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))), "pmg_level_dx")
        return out

    def epw(self):
        """``pmg_level_epw``: (current elements per workgroup of the fused kernel, compiled candidates)."""
        cur, n = C.c_int32(0), C.c_int32(0)
        cand = (C.c_int32 * 4)()
        A.check(A.lib().pmg_level_epw(self.handle, C.byref(cur), cand, C.byref(n)), "pmg_level_epw")
        return cur.value, [cand[i] for i in range(n.value)]

    def set_epw(self, epw: int) -> None:
        """``pmg_level_set_epw`` (0: the default for P)."""
        A.check(A.lib().pmg_level_set_epw(self.handle, int(epw)), "pmg_level_set_epw")

    def autotune(self, precision: int = 32, reps: int = 10, stream=None) -> dict:
        """``pmg_level_autotune``: time every candidate, keep the fastest; returns
        {"epw": chosen, "us_per_residual_and_sweep": {candidate: microseconds}}."""
        _, cand = self.epw()
        us = (C.c_double * 4)()
        best = C.c_int32(0)
        A.check(A.lib().pmg_level_autotune(self.handle, precision, reps, C.byref(best), us, _stream(stream)),
                "pmg_level_autotune")
        return {"epw": best.value, "us_per_residual_and_sweep": {int(c): us[i] for i, c in enumerate(cand)}}

    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=torch.float64, device=self.torch_device)

    def status(self) -> int:
        flags = C.c_int32(0)
        A.check(A.lib().pmg_level_status(self.handle, C.byref(flags)), "pmg_level_status")
        return flags.value

    def check_state(self, t: torch.Tensor | None, name: str, allow_none: bool = True):
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.torch_device \
                or tuple(t.shape) != self.shape:
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {self.shape} on "
                             f"{self.torch_device}")
        return C.c_void_p(t.data_ptr())

    def close(self):
        if getattr(self, "handle", None):
            A.lib().pmg_level_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factors:
    """Inverse element blocks of one level (a ``pmg_factors`` handle)."""

    def __init__(self, level: Level, precision: int = 64):
        h = A.pmg_factors()
        A.check(A.lib().pmg_factors_create(level.handle, precision, C.byref(h)), "pmg_factors_create")
        self.handle = h
        self.level = level
        self.precision = precision

    def close(self):
        if getattr(self, "handle", None):
            A.lib().pmg_factors_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LineFactors(Factors):
    """Element-line Jacobi blocks of one level (a ``pmg_factors`` handle made by
    ``pmg_line_factors_create``); ``lines`` is an [n_lines, K] integer array of element indices in
    line order covering every element once."""

    def __init__(self, level: Level, lines, precision: int = 64):
        import numpy as np
        arr = np.ascontiguousarray(np.asarray(lines), dtype=np.int32)
        if arr.ndim != 2:
            raise ValueError("lines must be a 2-D array [n_lines, K]")
        h = A.pmg_factors()
        A.check(A.lib().pmg_line_factors_create(level.handle, precision, arr.ctypes.data_as(C.POINTER(C.c_int32)),
                                                 arr.shape[0], arr.shape[1], C.byref(h)), "pmg_line_factors_create")
        self.handle = h
        self.level = level
        self.precision = precision
        self.lines = arr


def line_blocks(fac: LineFactors, q, dtau: float, c_mass: float = 0.0, stream=None):
    """Refactor the line factors at state q and return (D, Am, Ap), each [Ne, n, n] float64 on the
    level's device (row index p*Nv + v; Am/Ap the blocks towards the previous/next element of the
    line, zero at the line's ends)."""
    lev = fac.level
    shape = (lev.ne, lev.n, lev.n)
    D, Am, Ap = (torch.empty(shape, dtype=torch.float64, device=lev.torch_device) for _ in range(3))
    A.check(A.lib().pmg_line_blocks(fac.handle, lev.check_state(q, "q", False), dtau, c_mass,
                                    C.c_void_p(D.data_ptr()), C.c_void_p(Am.data_ptr()), C.c_void_p(Ap.data_ptr()),
                                    _stream(stream)), "pmg_line_blocks")
    return D, Am, Ap


def _norms_ptr(level: Level, norms):
    if norms is None:
        return None
    if norms.dtype != torch.float64 or norms.numel() < level.nv + 1 or norms.device != level.torch_device:
        raise ValueError("norms must be a float64 device tensor with Nv+1 entries")
    return C.c_void_p(norms.data_ptr())


def fr_residual(level: Level, q, F, src=None, S=None, c_mass: float = 0.0, norms=None, stream=None):
    A.check(A.lib().fr_residual(level.handle, level.check_state(q, "q", False), level.check_state(src, "src"),
                                level.check_state(S, "S"), c_mass, level.check_state(F, "F", False),
                                _norms_ptr(level, norms), _stream(stream)), "fr_residual")


def fr_residual_noalloc(level: Level, q, F, src=None, S=None, c_mass: float = 0.0, norms=None, stream=None):
    """fr_residual whose norm partials live in the library's static device scratch (the C entry
    point allocates nothing)."""
    A.check(A.lib().fr_residual_noalloc(level.handle, level.check_state(q, "q", False),
                                        level.check_state(src, "src"), level.check_state(S, "S"), c_mass,
                                        level.check_state(F, "F", False), _norms_ptr(level, norms),
                                        _stream(stream)), "fr_residual_noalloc")


def fr_conservative(level: Level, q, qc, stream=None):
    A.check(A.lib().fr_conservative(level.handle, level.check_state(q, "q", False),
                                    level.check_state(qc, "qc", False), _stream(stream)), "fr_conservative")


def fr_element_jacobian(level: Level, q, dtau: float, c_mass: float, factors: Factors, D_out=None, stream=None):
    dptr = None
    if D_out is not None:
        if D_out.dtype != torch.float64 or not D_out.is_contiguous() or D_out.numel() != level.ne * level.n ** 2:
            raise ValueError("D_out must be a contiguous float64 tensor with Ne*n*n entries")
        dptr = C.c_void_p(D_out.data_ptr())
    A.check(A.lib().fr_element_jacobian(level.handle, level.check_state(q, "q", False), dtau, c_mass, dptr,
                                        factors.handle, _stream(stream)), "fr_element_jacobian")


def ejacobi_sweep(level: Level, factors: Factors, q, n_sweeps: int, src=None, S=None, c_mass: float = 0.0,
                  alpha_r: float = 1.0, F_after=None, norms=None, stream=None):
    A.check(A.lib().ejacobi_sweep(level.handle, factors.handle, level.check_state(q, "q", False),
                                  level.check_state(src, "src"), level.check_state(S, "S"), c_mass, n_sweeps,
                                  alpha_r, level.check_state(F_after, "F_after"), _norms_ptr(level, norms),
                                  _stream(stream)), "ejacobi_sweep")


def pmg_restrict(fine: Level, coarse: Level, x_f, x_c, nvar: int | None = None, stream=None):
    """x_c = restriction of x_f (all Nv variables unless nvar is given)."""
    nvar = fine.nv if nvar is None else nvar
    A.check(A.lib().pmg_restrict(fine.handle, coarse.handle, fine.check_state(x_f, "x_f", False),
                                 coarse.check_state(x_c, "x_c", False), nvar, _stream(stream)), "pmg_restrict")


def pmg_prolong(coarse: Level, fine: Level, dx_c, x_f, nvar: int | None = None, stream=None):
    """x_f += prolongation of dx_c (all Nv variables unless nvar is given)."""
    nvar = fine.nv if nvar is None else nvar
    A.check(A.lib().pmg_prolong(coarse.handle, fine.handle, coarse.check_state(dx_c, "dx_c", False),
                                fine.check_state(x_f, "x_f", False), nvar, _stream(stream)), "pmg_prolong")


class StageSolver:
    """Holds the levels, factors and options of ``esdirk_stage_solve``."""

    def __init__(self, levels, factors, n_smooth, *, dtau_init=0.01, dtau_max=10.0, ser_exponent=1.5,
                 refresh_every=10, freeze_at_max=True, tol_rel=1e-8, max_vcycles=200, alpha_r=1.0,
                 use_graph=False, use_cfl=False, cfl_init=1e2, cfl_max=1e5, stage_guess="previous",
                 ser_floor=False, lookahead=1):
        self.levels = list(levels)
        self.factors = list(factors)
        nl = len(self.levels)
        self._lh = (A.pmg_level * nl)(*[lv.handle for lv in self.levels])
        self._fh = (A.pmg_factors * nl)(*[f.handle for f in self.factors])
        self._ns = (C.c_int32 * nl)(*n_smooth)
        o = A.SolveOpts()
        o.n_levels, o.levels, o.factors, o.n_smooth = nl, self._lh, self._fh, self._ns
        o.dtau_init, o.dtau_max, o.ser_exponent = dtau_init, dtau_max, ser_exponent
        o.refresh_every, o.freeze_at_max, o.tol_rel = refresh_every, int(freeze_at_max), tol_rel
        o.max_vcycles, o.alpha_r = max_vcycles, alpha_r
        o.use_graph = int(use_graph)
        o.use_cfl, o.cfl_init, o.cfl_max = int(use_cfl), cfl_init, cfl_max
        o.stage_guess = {"previous": 0, "predictor": 1}[stage_guess]   # used by esdirk_step
        o.ser_floor = int(ser_floor)
        if lookahead not in (0, 1, 2):
            raise ValueError("lookahead must be 0 (off), 1 (on) or 2 (always, for tests)")
        o.lookahead = int(lookahead)
        self.opts = o

    def solve(self, q, *, omega=0.0, dt=0.0, qc_n=None, R_prev=(), a_row=(), R_out=None, stream=None,
              raise_on_error=True):
        L0 = self.levels[0]
        nprev = len(R_prev)
        rp = (C.c_void_p * max(nprev, 1))(*[L0.check_state(r, "R_prev", False) for r in R_prev])
        ar = (C.c_double * max(nprev, 1))(*a_row)
        cap = self.opts.max_vcycles + 1
        hist = (C.c_double * cap)()
        st = A.SolveStats()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_capacity = cap
        status = A.lib().esdirk_stage_solve(C.byref(self.opts), omega, dt, L0.check_state(qc_n, "qc_n"), rp, ar,
                                            nprev, L0.check_state(q, "q", False), L0.check_state(R_out, "R_out"),
                                            C.byref(st), _stream(stream))
        out = {"status": status, "n_vcycles": st.n_vcycles, "n_refresh": st.n_refresh, "r0": st.r0,
               "r_final": st.r_final, "seconds": st.seconds, "dtau_min": st.dtau_min,
               "history": list(hist[:min(st.n_vcycles + 1, cap)])}
        if raise_on_error:
            A.check(status, "esdirk_stage_solve")
        return out


def nk_stage_solve(solver: StageSolver, q, *, krylov_dim=10, eta=1e-2, max_newton=50, fd_rel=1e-3, pc_rel=1e-3,
                   precondition=True, omega=0.0, dt=0.0, qc_n=None, R_prev=(), a_row=(), work=None, stream=None,
                   raise_on_error=True):
    """``nk_stage_solve``: Newton-Krylov stage solve with the solver's V-cycle as preconditioner
    (levels, factors, smoothing counts, dtau/CFL range, SER and refresh rule from ``solver``;
    ``tol_rel`` from it too). ``fd_rel`` and ``pc_rel`` are RMS perturbations per state entry
    (about sqrt(machine epsilon) times the absolute state: the defaults suit pressures near 1e4-1e5).
    ``work``: a float64 device tensor of at least ``nk_work_elems`` entries (allocated here when
    None). Returns the stats dict with ``n_newton`` and ``n_krylov``."""
    L0 = solver.levels[0]
    need = int(A.lib().nk_work_elems(L0.handle, krylov_dim))
    if need < 0:
        raise ValueError("krylov_dim must be in 1..32")
    if work is None:
        work = torch.empty(need, dtype=torch.float64, device=L0.torch_device)
    if work.dtype != torch.float64 or not work.is_contiguous() or work.numel() < need or work.device != L0.torch_device:
        raise ValueError(f"work must be a contiguous float64 tensor of at least {need} entries on the level's device")
    nk = A.NkOpts(krylov_dim, max_newton, eta, fd_rel, pc_rel, 1 if precondition else 0)
    nprev = len(R_prev)
    rp = (C.c_void_p * max(nprev, 1))(*[L0.check_state(r, "R_prev", False) for r in R_prev])
    ar = (C.c_double * max(nprev, 1))(*a_row)
    cap = max_newton + 1
    hist = (C.c_double * cap)()
    st = A.SolveStats()
    st.history = C.cast(hist, C.POINTER(C.c_double))
    st.history_capacity = cap
    nkry = C.c_int32(0)
    status = A.lib().nk_stage_solve(C.byref(solver.opts), C.byref(nk), omega, dt, L0.check_state(qc_n, "qc_n"), rp,
                                    ar, nprev, L0.check_state(q, "q", False), C.c_void_p(work.data_ptr()), C.byref(st),
                                    C.byref(nkry), _stream(stream))
    out = {"status": status, "n_newton": st.n_vcycles, "n_krylov": nkry.value, "n_refresh": st.n_refresh,
           "r0": st.r0, "r_final": st.r_final, "seconds": st.seconds, "dtau_min": st.dtau_min,
           "history": list(hist[:min(st.n_vcycles + 1, cap)])}
    if raise_on_error:
        A.check(status, "nk_stage_solve")
    return out


def dtau_min(level: Level, q, stream=None) -> float:
    """``pmg_dtau_min``: the pseudo-time scale of eq. (33) at state q (synchronises)."""
    out = C.c_double(0.0)
    A.check(A.lib().pmg_dtau_min(level.handle, level.check_state(q, "q", False), C.byref(out), _stream(stream)),
            "pmg_dtau_min")
    return out.value


def esdirk_stages(scheme: int) -> int:
    return int(A.lib().esdirk_stages(scheme))


def esdirk_butcher(scheme: int):
    """The library's Butcher matrix of an ESDIRK scheme id (s x s numpy array)."""
    import numpy as np
    s = esdirk_stages(scheme)
    if s == 0:
        raise ValueError(f"unknown ESDIRK scheme {scheme}")
    buf = (C.c_double * (s * s))()
    A.lib().esdirk_butcher(scheme, buf)
    return np.array(buf[:], dtype=float).reshape(s, s)


def esdirk_step(solver: StageSolver, scheme: int, dt: float, q, work, stream=None, raise_on_error=True):
    """One time step of ``esdirk_step``; ``work`` is a float64 device tensor of shape
    (stages, Nv, Np, Ne). Returns one stats dict per implicit stage (with its residual history)."""
    L0 = solver.levels[0]
    s = esdirk_stages(scheme)
    if s == 0:
        raise ValueError(f"unknown ESDIRK scheme {scheme}")
    if work.dtype != torch.float64 or not work.is_contiguous() or tuple(work.shape) != (s,) + L0.shape \
            or work.device != L0.torch_device:
        raise ValueError(f"work must be a contiguous float64 tensor of shape {(s,) + L0.shape}")
    stats = (A.SolveStats * (s - 1))()
    cap = solver.opts.max_vcycles + 1
    hists = [(C.c_double * cap)() for _ in range(s - 1)]
    for st, h in zip(stats, hists):
        st.history = C.cast(h, C.POINTER(C.c_double))
        st.history_capacity = cap
    status = A.lib().esdirk_step(C.byref(solver.opts), scheme, dt, L0.check_state(q, "q", False),
                                 C.c_void_p(work.data_ptr()), stats, s - 1, _stream(stream))
    out = [{"status": st.status, "n_vcycles": st.n_vcycles, "n_refresh": st.n_refresh, "r0": st.r0,
            "r_final": st.r_final, "seconds": st.seconds, "dtau_min": st.dtau_min,
            "history": list(h[:min(st.n_vcycles + 1, cap)])} for st, h in zip(stats, hists)]
    if raise_on_error:
        A.check(status, "esdirk_step")
    return out


class Batch:
    """Independent cases advanced together (a ``pmg_batch``): each case is a StageSolver (its own
    levels, factors and options); the library runs them concurrently, one stream per case."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        n = len(self.solvers)
        self._opts = (A.SolveOpts * n)(*[sv.opts for sv in self.solvers])
        h = A.pmg_batch()
        A.check(A.lib().pmg_batch_create(self._opts, n, C.byref(h)), "pmg_batch_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            A.lib().pmg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def esdirk_step(self, scheme: int, dt, q, work, stream=None, raise_on_error=True):
        """One ESDIRK time step of every case: dt a sequence (one per case), q and work lists of
        device tensors (work[c] of shape (stages, Nv, Np, Ne) of case c). Returns, per case, one
        stats dict per implicit stage."""
        n = len(self.solvers)
        s = esdirk_stages(scheme)
        if s == 0:
            raise ValueError(f"unknown ESDIRK scheme {scheme}")
        qp = (C.c_void_p * n)(*[sv.levels[0].check_state(x, "q", False) for sv, x in zip(self.solvers, q)])
        for sv, w in zip(self.solvers, work):
            L0 = sv.levels[0]
            if w.dtype != torch.float64 or not w.is_contiguous() or tuple(w.shape) != (s,) + L0.shape \
                    or w.device != L0.torch_device:
                raise ValueError(f"work must be a contiguous float64 tensor of shape {(s,) + L0.shape}")
        wp = (C.c_void_p * n)(*[w.data_ptr() for w in work])
        dts = (C.c_double * n)(*dt)
        stats = (A.SolveStats * (n * (s - 1)))()
        hists = []
        for c, sv in enumerate(self.solvers):
            cap = sv.opts.max_vcycles + 1
            for i in range(s - 1):
                h = (C.c_double * cap)()
                hists.append(h)
                st = stats[c * (s - 1) + i]
                st.history = C.cast(h, C.POINTER(C.c_double))
                st.history_capacity = cap
        status = A.lib().esdirk_step_batched(self.handle, scheme, dts, qp, wp, stats, _stream(stream))
        out = []
        for c, sv in enumerate(self.solvers):
            cap = sv.opts.max_vcycles + 1
            per = []
            for i in range(s - 1):
                st, h = stats[c * (s - 1) + i], hists[c * (s - 1) + i]
                per.append({"status": st.status, "n_vcycles": st.n_vcycles, "n_refresh": st.n_refresh,
                            "r0": st.r0, "r_final": st.r_final, "seconds": st.seconds,
                            "history": list(h[:min(st.n_vcycles + 1, cap)])})
            out.append(per)
        if raise_on_error:
            A.check(status, "esdirk_step_batched")
        return out

    def solve(self, q, omega=None, dt=None, qc_n=None, R_prev=None, a_row=None, R_out=None, stream=None,
              raise_on_error=True):
        """esdirk_stage_solve_batched; every argument but q is a per-case list (dt[c] <= 0 or None:
        steady case c)."""
        n = len(self.solvers)
        dt = [0.0] * n if dt is None else [0.0 if d is None else d for d in dt]
        omega = [0.0] * n if omega is None else list(omega)
        L0s = [sv.levels[0] for sv in self.solvers]
        qp = (C.c_void_p * n)(*[L.check_state(x, "q", False) for L, x in zip(L0s, q)])
        qcp = (C.c_void_p * n)(*[(L.check_state(qc_n[c], "qc_n") if qc_n and qc_n[c] is not None else None)
                                for c, L in enumerate(L0s)])
        keep = []
        rpp = (C.POINTER(C.c_void_p) * n)()
        arp = (C.POINTER(C.c_double) * n)()
        npv = (C.c_int32 * n)()
        for c, L in enumerate(L0s):
            rs = R_prev[c] if R_prev and R_prev[c] else []
            arr = (C.c_void_p * max(len(rs), 1))(*[L.check_state(r, "R_prev", False) for r in rs])
            av = (C.c_double * max(len(rs), 1))(*(a_row[c] if a_row and a_row[c] else []))
            keep += [arr, av]
            rpp[c] = C.cast(arr, C.POINTER(C.c_void_p))
            arp[c] = C.cast(av, C.POINTER(C.c_double))
            npv[c] = len(rs)
        rop = (C.c_void_p * n)(*[(L.check_state(R_out[c], "R_out") if R_out and R_out[c] is not None else None)
                                for c, L in enumerate(L0s)])
        stats = (A.SolveStats * n)()
        hists = []
        for c, sv in enumerate(self.solvers):
            h = (C.c_double * (sv.opts.max_vcycles + 1))()
            hists.append(h)
            stats[c].history = C.cast(h, C.POINTER(C.c_double))
            stats[c].history_capacity = sv.opts.max_vcycles + 1
        status = A.lib().esdirk_stage_solve_batched(self.handle, (C.c_double * n)(*omega), (C.c_double * n)(*dt),
                                                    qcp, rpp, arp, npv, qp, rop, stats, _stream(stream))
        out = [{"status": st.status, "n_vcycles": st.n_vcycles, "n_refresh": st.n_refresh, "r0": st.r0,
                "r_final": st.r_final, "seconds": st.seconds, "dtau_min": st.dtau_min,
                "history": list(h[:min(st.n_vcycles + 1, len(h))])} for st, h in zip(stats, hists)]
        if raise_on_error:
            A.check(status, "esdirk_stage_solve_batched")
        return out
