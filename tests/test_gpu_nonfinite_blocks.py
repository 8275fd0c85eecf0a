"""Block rebuilds from a state holding a NaN, for every elimination kernel family: the level's fault
flag is raised (the eliminations replace a non-finite or zero pivot by 1 and carry on, so every
workgroup runs to its end and writes only inside the factor store), and a rebuild from the clean
state afterwards gives blocks whose sweep is finite with no fault.

Kernels covered: the 2-D register-row elimination (P4 FP64), the 2-D block-in-LDS FP32 elimination
(P4 FP32), the 3-D register-row elimination (P2 FP64), the 3-D block-in-LDS FP32 elimination (P2
FP32) and the 3-D large-block elimination through global work slots (P3, FP32 and FP64)."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_03972_amd import _abi as A  # noqa: E402
from paper_1908_03972_amd import api  # noqa: E402

FS2 = W.FreeStreamSpec()
FS3 = W.FreeStream3Spec(ma_inf=0.01)


def level(dim, P):
    if dim == 2:
        mesh, fs = W.airfoil_o_mesh(16, 8, ratio=1.3, r_far=10.0), FS2
    else:
        mesh, fs = W.cubed_sphere_mesh(2, 2), FS3
    qinf = fs.freestream()
    return mesh, api.Level(mesh, P, gamma=fs.gamma, rgas=fs.rgas, eps_mode=1, ma_inf=fs.ma_inf, kappa=1.0,
                           q_inf=qinf, q_ref=qinf)


@pytest.mark.parametrize("dim,P,prec", [(2, 4, 64), (2, 4, 32), (3, 2, 64), (3, 2, 32), (3, 3, 32), (3, 3, 64)])
def test_rebuild_from_a_nan_state_flags_and_recovers(dim, P, prec):
    mesh, lv = level(dim, P)
    fac = api.Factors(lv, prec)
    q = lv.new_state()                       # the free stream (zero offset)
    dtau = 10.0 * api.dtau_min(lv, q)
    api.fr_element_jacobian(lv, q, dtau, 0.0, fac)
    torch.cuda.synchronize()
    assert lv.status() == 0
    bad = q.clone()
    bad[0, 0, 0] = float("nan")              # variable 0, point 0 of element 0
    api.fr_element_jacobian(lv, bad, dtau, 0.0, fac)
    torch.cuda.synchronize()
    with pytest.raises(A.PmgError) as err:   # the flag is read (and cleared) as PMG_E_SINGULAR
        lv.status()
    assert err.value.status == A.PMG_E_SINGULAR
    # a sweep with the clean state and the rebuilt (clean) blocks is finite again
    api.fr_element_jacobian(lv, q, dtau, 0.0, fac)
    torch.cuda.synchronize()
    assert lv.status() == 0
    qs = q.clone()
    api.ejacobi_sweep(lv, fac, qs, 1)
    torch.cuda.synchronize()
    assert lv.status() == 0
    assert bool(torch.isfinite(qs).all())
