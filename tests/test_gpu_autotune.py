"""Elements per workgroup of the fused residual / element-Jacobi kernel on quadrilateral levels:
every compiled variant gives the default variant's residual and sweep (the per-element arithmetic
does not depend on how elements are grouped; the residual norms differ only in their summation
order), and the tuner keeps one of the candidates. 7 x 7 jittered periodic mesh: 49 elements, so
every candidate has a ragged last workgroup."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402

pytestmark = pytest.mark.gpu


def setup(P):
    mesh = W.periodic_quad_mesh(7, 10.0, jitter=0.1, seed=W.JITTER_SEED)
    vs = W.VortexSpec(length=10.0)
    qinf = vs.freestream()
    lev = api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf, q_inf=qinf, q_ref=qinf)
    x, y = lev.points()
    q = torch.from_numpy(np.ascontiguousarray(np.moveaxis(vs.state(x, y) - qinf, -1, 0))).cuda()
    return lev, q


def run(lev, q, fac, c_mass):
    F = lev.new_state()
    nr = torch.zeros(lev.nv + 1, dtype=torch.float64, device=q.device)
    api.fr_residual(lev, q, F, c_mass=c_mass, norms=nr)
    qs = q.clone()
    ns = torch.zeros(lev.nv + 1, dtype=torch.float64, device=q.device)
    Fa = lev.new_state()
    api.ejacobi_sweep(lev, fac, qs, 2, c_mass=c_mass, F_after=Fa, norms=ns)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (F, nr, qs, ns, Fa)]


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("prec", [32, 64])
def test_every_variant_matches_the_default(P, prec):
    lev, q = setup(P)
    cur, cand = lev.epw()
    assert cur == cand[0] and len(cand) >= 2
    c_mass = 1.0 / (0.05 * (1.0 - 2.0 ** -0.5))
    fac = api.Factors(lev, prec)
    api.fr_element_jacobian(lev, q, 0.05, c_mass, fac)
    ref = run(lev, q, fac, c_mass)
    for epw in cand[1:]:
        lev.set_epw(epw)
        assert lev.epw()[0] == epw
        got = run(lev, q, fac, c_mass)
        print("P", P, "prec", prec, "epw", epw)
        for name, g, r in zip(("F", "norms", "q after sweeps", "sweep norms", "F after"), got, ref):
            if "norms" in name:
                np.testing.assert_allclose(g, r, rtol=1e-13, atol=0.0, err_msg=name)
            else:
                assert np.array_equal(g, r), (name, float(np.max(np.abs(g - r))))
    lev.set_epw(0)
    assert lev.epw()[0] == cand[0]


@pytest.mark.parametrize("P", [1, 3])
def test_autotune_keeps_a_candidate(P):
    lev, q = setup(P)
    _, cand = lev.epw()
    res = lev.autotune(precision=32, reps=3)
    assert res["epw"] in cand
    assert lev.epw()[0] == res["epw"]
    assert sorted(res["us_per_residual_and_sweep"]) == sorted(cand)
    assert all(v > 0.0 for v in res["us_per_residual_and_sweep"].values())
    assert lev.status() == 0
    # results after tuning still equal the default variant's
    c_mass = 2.0
    fac = api.Factors(lev, 64)
    api.fr_element_jacobian(lev, q, 0.05, c_mass, fac)
    got = run(lev, q, fac, c_mass)
    lev.set_epw(0)
    ref = run(lev, q, fac, c_mass)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])


def test_set_epw_rejects_uncompiled_values():
    lev, _ = setup(2)
    with pytest.raises(api.A.PmgError):
        lev.set_epw(5)
    with pytest.raises(api.A.PmgError):
        lev.autotune(precision=16)


# hexahedral levels: the rotated 3 x 3 x 2 cubed sphere (108 elements, every face orientation code)

def setup3(P):
    from test_gpu_3d import disturbed_at
    from test_oracle_3d import small_sphere
    fs = W.FreeStream3Spec(ma_inf=0.01)
    qinf = fs.freestream()
    lev = api.Level(small_sphere(inner=W.BC_SLIP_WALL), P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1,
                    ma_inf=fs.ma_inf, kappa=1.0, q_inf=qinf, q_ref=qinf)
    x = np.moveaxis(np.asarray(lev.points()), 0, -1)
    q = torch.from_numpy(np.ascontiguousarray(np.moveaxis(disturbed_at(x, qinf) - qinf, -1, 0))).cuda()
    return lev, q


@pytest.mark.parametrize("P", [0, 1, 2, 3])
def test_every_3d_variant_matches_the_default(P):
    lev, q = setup3(P)
    cur, cand = lev.epw()
    assert cur == cand[0] and len(cand) >= 2
    fac = api.Factors(lev, 32)
    dtau = 0.2 * api.dtau_min(lev, q)
    api.fr_element_jacobian(lev, q, dtau, 0.0, fac)
    ref = run(lev, q, fac, 0.0)
    for epw in cand[1:]:
        lev.set_epw(epw)
        got = run(lev, q, fac, 0.0)
        print("3-D P", P, "epw", epw)
        for name, g, r in zip(("F", "norms", "q after sweeps", "sweep norms", "F after"), got, ref):
            if "norms" in name:
                np.testing.assert_allclose(g, r, rtol=1e-13, atol=0.0, err_msg=name)
            else:
                assert np.array_equal(g, r), (name, float(np.max(np.abs(g - r))))
    res = lev.autotune(precision=32, reps=2)
    assert res["epw"] in cand and lev.status() == 0
