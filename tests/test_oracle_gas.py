"""Pins of the oracle's physics: M, A_n, Gamma, the eigen-system and the common flux."""
import numpy as np
import pytest

from oracle import gas as G

GAS = G.Gas(eps_mode="local")


def _state(rng, n=16, d=2):
    p = 57142.857 * (1 + 0.01 * rng.standard_normal(n))
    u = rng.standard_normal((n, d))
    T = 57142.857 * (1 + 0.01 * rng.standard_normal(n))
    return np.concatenate([p[:, None], u, T[:, None]], axis=1)


def _cstep(fun, q, h=1e-30):
    """Complex-step Jacobian of fun w.r.t. the last axis of q."""
    nv = q.shape[-1]
    cols = []
    for c in range(nv):
        qc = q.astype(complex)
        qc[..., c] += 1j * h
        cols.append(fun(qc).imag / h)
    return np.stack(cols, axis=-1)


@pytest.mark.parametrize("d", [2, 3])
def test_mass_matrix_is_dqc_dqp(d):
    q = _state(np.random.default_rng(0), d=d)
    M = G.mass_matrix(q, GAS)
    Mcs = _cstep(lambda x: G.conservative(x, GAS), q)
    rowscale = np.max(np.abs(Mcs), axis=-1, keepdims=True)
    assert np.max(np.abs(M - Mcs) / rowscale) < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_flux_jacobian_is_dfn_dqp(d):
    rng = np.random.default_rng(1)
    q = _state(rng, d=d)
    n = rng.standard_normal((q.shape[0], d))
    A = G.flux_jacobian(q, n, GAS)
    Acs = _cstep(lambda x: G.normal_flux(x, n, GAS), q)
    assert np.max(np.abs(A - Acs)) <= 1e-13 * np.max(np.abs(Acs))


@pytest.mark.parametrize("d", [2, 3])
def test_gamma_equals_M_when_ur_is_c(d):
    q = _state(np.random.default_rng(2), d=d)
    gam = G.preconditioner(q, GAS, eps=np.ones(q.shape[0]))
    M = G.mass_matrix(q, GAS)
    rowscale = np.max(np.abs(M), axis=-1, keepdims=True)
    assert np.max(np.abs(gam - M) / rowscale) < 1e-14


def test_beta_is_inverse_c_squared():
    q = _state(np.random.default_rng(3))
    p, T = q[:, 0], q[:, -1]
    rho = G.density(q, GAS)
    beta = 1 / (GAS.rgas * T) + (-p / (GAS.rgas * T * T)) / (rho * GAS.cp)
    assert np.allclose(beta * G.sound_speed(q, GAS) ** 2, 1.0, rtol=1e-14)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("mode", ["local", "unit"])
def test_eigenvalues_match_numerical_spectrum(d, mode):
    rng = np.random.default_rng(4)
    q = _state(rng, d=d)
    n = rng.standard_normal((q.shape[0], d))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    eps = None if mode == "local" else np.ones(q.shape[0])
    gam = G.preconditioner(q, GAS, eps)
    X = np.linalg.solve(gam, G.flux_jacobian(q, n, GAS))
    ev = np.sort(np.linalg.eigvals(X).real, axis=1)
    l1, l2, l3 = G.preconditioned_eigenvalues(q, n, GAS, eps)
    ref = np.sort(np.stack([l1] * d + [l2, l3], axis=1), axis=1)
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    assert np.max(np.abs(ev - ref) / scale) < 1e-10
    if mode == "unit":   # unpreconditioned: u_n, u_n +- c
        c = G.sound_speed(q, GAS)
        un = np.sum(q[:, 1:-1] * n, axis=1)
        assert np.allclose(l2, un + c, rtol=1e-13) and np.allclose(l3, un - c, rtol=1e-13)


def _abs_matrix_eig(X):
    w, V = np.linalg.eig(X)
    return (V * np.abs(w.real)[..., None, :]) @ np.linalg.inv(V)


def test_common_flux_dissipation_matches_eigendecomposition():
    rng = np.random.default_rng(5)
    qm = _state(rng)
    qp = qm * (1 + 1e-3 * rng.standard_normal(qm.shape))
    S = rng.standard_normal((qm.shape[0], 2))
    n = S / np.linalg.norm(S, axis=1, keepdims=True)
    qa = 0.5 * (qm + qp)
    gam = G.preconditioner(qa, GAS)
    X = np.linalg.solve(gam, G.flux_jacobian(qa, n, GAS))
    diss = (gam @ (_abs_matrix_eig(X) @ (qp - qm)[..., None]))[..., 0].real
    ref = np.linalg.norm(S, axis=1)[:, None] * (
        0.5 * (G.normal_flux(qm, n, GAS) + G.normal_flux(qp, n, GAS)) - 0.5 * diss)
    got = G.common_flux(qm, qp, S, GAS)
    assert np.max(np.abs(got - ref) / np.max(np.abs(ref), axis=0)) < 1e-11


def test_common_flux_consistency_and_conservation():
    rng = np.random.default_rng(6)
    a = _state(rng, d=3)
    b = a * (1 + 1e-2 * rng.standard_normal(a.shape))
    S = rng.standard_normal((a.shape[0], 3))
    fa = G.normal_flux(a, S, GAS)
    assert np.max(np.abs(G.common_flux(a, a, S, GAS) - fa) / np.max(np.abs(fa), axis=0)) < 1e-13
    lhs = G.common_flux(a, b, S, GAS)
    rhs = -G.common_flux(b, a, -S, GAS)
    assert np.max(np.abs(lhs - rhs) / np.max(np.abs(lhs), axis=0)) < 1e-12


def test_common_flux_is_upwind_for_supersonic_unpreconditioned_flow():
    """With eps = 1 (Gamma = M) and all eigenvalues positive, f_com(a, b) - f(a) = O(|b-a|^2)."""
    gas = G.Gas(eps_mode="cutoff", ma_inf=2.0, kappa=1.0)   # eps = min(1, max(2, Ma)) = 1
    a = np.array([[1.0, 3.0, 0.2, 1.0]])                     # c = sqrt(1.4) ~ 1.18 < u = 3
    S = np.array([[1.0, 0.0]])
    dirn = np.array([[0.3, -0.5, 0.7, 0.2]])
    errs = []
    for h in (1e-3, 5e-4):
        b = a + h * dirn
        errs.append(np.max(np.abs(G.common_flux(a, b, S, gas) - G.normal_flux(a, S, gas))))
    assert errs[0] / errs[1] > 3.5      # second order in the jump
    b = a + 1e-3 * dirn                  # the downwind-weighted mean would be first order
    assert np.max(np.abs(G.common_flux(a, b, S, gas) - G.normal_flux(b, S, gas))) > 10 * errs[0]


def _mach_state(ma, c=100.0, d=2, gas=GAS):
    """Primitive states (p, u, T) of sound speed c (T = c^2 / (gamma R)) and speed |u| = ma c,
    the velocity along a fixed oblique direction."""
    T = c * c / (gas.gamma * gas.rgas)
    ma = np.asarray(ma, float)
    direction = np.array([0.6, 0.8]) if d == 2 else np.array([2.0, -3.0, 6.0]) / 7.0
    u = (ma * c)[:, None] * direction[None, :]
    return np.concatenate([np.full((ma.size, 1), 1.0e4), u, np.full((ma.size, 1), T)], axis=1)


@pytest.mark.parametrize("d", [2, 3])
def test_epsilon_closed_form(d):
    """Eq. (11): eps = min(1, max(kappa Ma_inf, Ma)) with the cut-off, eps = min(1, Ma) without
    (Sec. 4.1), and U_r = eps c in Theta of eq. (10). The states have Ma = |u|/c exactly; with
    kappa = 2, Ma_inf = 0.01 the cut-off is 0.02, so a swapped min/max, kappa applied to the
    local Mach number (max(Ma_inf, kappa Ma) = 0.03 at Ma = 0.015) or the cut-off applied in the
    local mode all fail."""
    ma = np.array([5e-4, 0.015, 0.02, 0.3, 0.999, 1.0, 2.0])
    q = _mach_state(ma, d=d)
    local = G.Gas(eps_mode="local")
    cut = G.Gas(eps_mode="cutoff", ma_inf=0.01, kappa=2.0)
    want_local = np.array([5e-4, 0.015, 0.02, 0.3, 0.999, 1.0, 1.0])
    want_cut = np.array([0.02, 0.02, 0.02, 0.3, 0.999, 1.0, 1.0])
    assert np.max(np.abs(G.epsilon(q, local) - want_local) / want_local) < 1e-14
    assert np.max(np.abs(G.epsilon(q, cut) - want_cut) / want_cut) < 1e-14
    # the reference velocity enters Gamma through Theta = 1/U_r^2 - rho_T/(rho C_p), U_r = eps c
    for gas, want in ((local, want_local), (cut, want_cut)):
        rho = q[:, 0] / (gas.rgas * q[:, -1])
        rho_T = -q[:, 0] / (gas.rgas * q[:, -1] ** 2)
        theta = 1.0 / (want * 100.0) ** 2 - rho_T / (rho * gas.cp)
        gam = G.preconditioner(q, gas)
        assert np.max(np.abs(gam[:, 0, 0] - theta) / theta) < 1e-13
