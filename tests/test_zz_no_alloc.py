"""fr_residual_noalloc (the stage residual with its norms, the norm partials in the library's static
device scratch) against fr_residual through the C ABI: F and the norms bit for bit, on two calls
in a row, the second on a smaller level, with a source, a forcing and a mass term; and the
rejection of a level whose norm partials exceed the scratch."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import api  # noqa: E402
from paper_1908_03972_amd import _abi as A  # noqa: E402


def _level(n, P, jitter):
    vs = W.VortexSpec()
    mesh = W.periodic_quad_mesh(n, 10.0, jitter=jitter, seed=W.JITTER_SEED)
    qinf = vs.freestream()
    lv = api.Level(mesh, P, gamma=vs.gamma, rgas=vs.rgas, eps_mode=0, ma_inf=vs.ma_inf, q_inf=qinf, q_ref=qinf)
    xy = lv.points()
    q = torch.from_numpy(np.ascontiguousarray(np.moveaxis(vs.state(xy[0], xy[1]) - qinf, -1, 0))).cuda()
    return lv, q


def test_noalloc_residual_matches_fr_residual_twice():
    rng = np.random.default_rng(9)
    for n, P in ((64, 3), (8, 2)):                      # the second call on a smaller level
        lv, q = _level(n, P, 0.1)
        print("fr_residual_noalloc on", n, "x", n, "P", P, flush=True)
        src = torch.from_numpy(rng.standard_normal(lv.shape)).cuda()
        S = torch.from_numpy(rng.standard_normal(lv.shape)).cuda()
        F_ref, F_na = lv.new_state(), lv.new_state()
        n_ref = torch.zeros(lv.nv + 1, dtype=torch.float64, device="cuda")
        n_na = torch.full((lv.nv + 1,), -1.0, dtype=torch.float64, device="cuda")
        api.fr_residual(lv, q, F_ref, src=src, S=S, c_mass=13.7, norms=n_ref)
        api.fr_residual_noalloc(lv, q, F_na, src=src, S=S, c_mass=13.7, norms=n_na)
        torch.cuda.synchronize()
        assert torch.equal(F_na, F_ref)
        assert torch.equal(n_na, n_ref), (n_na, n_ref)
        want = torch.linalg.vector_norm(F_ref.reshape(lv.nv, -1), dim=1)
        assert torch.allclose(n_na[:lv.nv], want, rtol=1e-13, atol=0.0)
        # without norms the call is fr_residual's residual
        F_nn = lv.new_state()
        api.fr_residual_noalloc(lv, q, F_nn, src=src, S=S, c_mass=13.7)
        torch.cuda.synchronize()
        assert torch.equal(F_nn, F_ref)


def test_noalloc_rejects_levels_beyond_its_scratch():
    # 400 x 400 elements at P3 with 8 elements per workgroup: 20000 workgroups x 4 variables of
    # partials, more than the 65536 doubles of the scratch
    lv, q = _level(400, 3, 0.0)
    lv.set_epw(8)
    F = lv.new_state()
    norms = torch.zeros(lv.nv + 1, dtype=torch.float64, device="cuda")
    st = A.lib().fr_residual_noalloc(lv.handle, q.data_ptr(), None, None, 0.0, F.data_ptr(), norms.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == A.PMG_E_ARG
    assert b"scratch" in A.lib().pmg_last_error()
    api.fr_residual(lv, q, F, norms=norms)             # the allocating entry point takes it
    torch.cuda.synchronize()
    assert float(norms[lv.nv]) > 0.0
