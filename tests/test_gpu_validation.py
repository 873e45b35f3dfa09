"""Validation of device inputs: a non-finite gamma never reaches the factorisation.

kf_set_gamma and kf_create with a device gamma count the NaN / inf entries with a
device reduction before anything is copied, and return KF_EINVAL; the problem keeps
its previous gamma and factors.  A finite gamma so large that omega^2 gamma overflows
builds blocks with infinite entries: the Gauss-Jordan pivot search of the
factorisation then meets columns with no finite entry, takes no interchange for them
(every index stays in range) and the solve reports a non-finite residual.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd._lib import KF_EINVAL, KF_ENAN, KFError  # noqa: E402
from paper_2204_06489_amd.solver import KKTProblem  # noqa: E402
from tests.oracle_cases import tiny_inputs  # noqa: E402


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_set_gamma_rejects_non_finite_and_keeps_state(bad):
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3)
    print(f"[case] set_gamma with a {bad} entry, 41x19 K=3", flush=True)
    p = KKTProblem.from_inputs(inp, eps=1.0)
    f = p.sources()
    u0, _ = p.helmholtz_solve(f)
    g_bad = torch.as_tensor(inp["gamma0"]).cuda().clone()
    g_bad[7, 11] = bad
    with pytest.raises(KFError) as e:
        p.set_gamma(g_bad)
    assert e.value.status == KF_EINVAL
    assert torch.equal(p.get_gamma().cpu(), torch.as_tensor(inp["gamma0"]))
    u1, _ = p.helmholtz_solve(f)        # the factors of the previous gamma still serve
    torch.cuda.synchronize()
    assert torch.equal(u0, u1)


def test_create_rejects_non_finite_device_gamma():
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3)
    g_bad = torch.as_tensor(inp["gamma0"]).cuda().clone()
    g_bad[-1, -1] = float("nan")
    with pytest.raises(KFError) as e:
        KKTProblem.from_inputs(inp, gamma=g_bad, eps=1.0)
    assert e.value.status == KF_EINVAL
    with pytest.raises(KFError) as e:
        KKTProblem.from_inputs(inp, gamma=g_bad.cpu().numpy(), eps=1.0)   # host path
    assert e.value.status == KF_EINVAL


def test_overflowing_gamma_gives_non_finite_solve_without_fault():
    """omega^2 gamma = inf at one node: the pivot guard keeps every index in range."""
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3)
    print("[case] overflowing gamma (1e308) through the FP64 factorisation, 41x19 K=3", flush=True)
    g = np.array(inp["gamma0"])
    g[9, 20] = 1e308
    p = KKTProblem.from_inputs(inp, gamma=torch.as_tensor(g).cuda(), eps=1.0)
    with pytest.raises(KFError) as e:
        p.helmholtz_solve(p.sources(), rtol=1e-12)
    torch.cuda.synchronize()
    assert e.value.status == KF_ENAN
    # a finite gamma afterwards factorises and solves normally again
    p.set_gamma(torch.as_tensor(inp["gamma0"]).cuda())
    x2, st2 = p.helmholtz_solve(p.sources(), rtol=1e-12)
    assert st2["rel_res_max"] <= 1e-12
