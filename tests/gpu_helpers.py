"""Shared helpers of the GPU parity tests: paired oracle / HIP levels on one seeded mesh, layout
conversion and the FP64 rounding floor used to state per-variable tolerances."""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle import gas as OG
from oracle.fr import FRLevel

PARITY_REL = 1e-11        # FP64 parity target: relative 2-norm per variable


def to_dev(x_epv, device="cuda"):
    """Oracle layout [Ne, Np, Nv] -> device layout [Nv, Np, Ne] (float64 tensor)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.transpose(x_epv, (2, 1, 0)))).to(device)


def from_dev(t):
    """Device layout [Nv, Np, Ne] -> oracle layout [Ne, Np, Nv] (numpy)."""
    return np.ascontiguousarray(np.transpose(t.detach().cpu().numpy(), (2, 1, 0)))


def gas_for(vs: W.VortexSpec, eps_mode="local"):
    return OG.Gas(gamma=vs.gamma, rgas=vs.rgas, eps_mode=eps_mode, ma_inf=vs.ma_inf)


def make_levels(mesh, P, vs: W.VortexSpec, device=0):
    from paper_1908_03972_amd import api
    gas = gas_for(vs)
    olev = FRLevel(mesh, P, gas, q_inf=vs.freestream())
    glev = api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf,
                     q_inf=vs.freestream(), q_ref=vs.freestream(), device=device)
    return olev, glev


def vortex_on(olev, vs):
    xy = olev.geo.xy
    return vs.state(xy[..., 0], xy[..., 1])


def rel_err_per_var(a, ref):
    """||a - ref||_2 / ||ref||_2 for each variable (last axis)."""
    num = np.linalg.norm((a - ref).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(ref.reshape(-1, ref.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def rounding_floor(fun, q, seed=1):
    """Relative change of fun(q) per variable when every entry of q moves by one unit in the last
    place: the size of the FP64 rounding noise the computation itself amplifies (cancellation in
    the preconditioned flux at low Mach number)."""
    rng = np.random.default_rng(seed)
    base = fun(q)
    pert = q * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=q.shape))
    return rel_err_per_var(fun(pert), base)


def tolerance(floor):
    """Per-variable parity bound: the FP64 target, or ten times the rounding floor where the
    method's own cancellation makes the target unreachable."""
    return np.maximum(PARITY_REL, 10.0 * floor)


def fp32_inverse(D):
    """Inverse of the block(s) D [..., n, n] computed in FP32: rows scaled by powers of two to a
    largest entry in [1/2, 1) (exact), the scaled block rounded to FP32 and inverted by LAPACK in
    FP32 with partial pivoting, the scales folded back. This reproduces the size of the error of an
    FP32 elimination (the GPU's mixed form) on the CPU; returned in FP64."""
    D = np.asarray(D, dtype=np.float64)
    mx = np.max(np.abs(D), axis=-1)
    s = np.ldexp(1.0, -np.frexp(np.where(mx > 0, mx, 1.0))[1])
    inv32 = np.linalg.inv((D * s[..., :, None]).astype(np.float32)).astype(np.float64)
    return inv32 * s[..., None, :]


def fp32_solver_class(fp32_elimination=False):
    """The oracle's PMG solver with the smoother's block inverses in FP32 and the block-vector
    products taken in FP32: the rounding the mixed-precision smoother introduces, reproduced on
    the CPU so that its effect sizes the FP32 parity tolerance (at Ma <= 1e-3 the temperature
    update amplifies it far beyond u_32). Where fp32_elimination holds (a bool, or a predicate on
    the level's P) the inverse itself is computed in FP32 (``fp32_inverse``, as the hexahedral
    blocks of P >= 2 are on the GPU); otherwise the FP64 inverse is rounded to FP32."""
    from oracle import solver as OS

    class PMGSolverFP32(OS.PMGSolver):
        def smooth(self, l, q, S, nsweep):
            lev = self.levels[l]
            elim = fp32_elimination(lev.P) if callable(fp32_elimination) else fp32_elimination
            if elim:
                winv = fp32_inverse(self.D[l]).astype(np.float32)
            else:
                winv = np.linalg.inv(self.D[l]).astype(np.float32)
            for _ in range(nsweep):
                Fq = self.F(l, q, S).reshape(lev.ne, lev.n, 1).astype(np.float32)
                dq = np.matmul(winv, Fq).astype(np.float64)
                q = q + self.opts.alpha_r * dq.reshape(q.shape)
            return q

    return PMGSolverFP32
