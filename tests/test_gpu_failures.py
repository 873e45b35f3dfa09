"""Failure handling of the Newton step, forced from the host (every kernel still ends
normally): an iteration limit that is too small returns KF_ENOCONV with the best
iterate and its statistics, a zero right-hand side returns xi = 0 after no
iteration, and non-finite data is reported as KF_ENAN."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd._lib import KF_ENAN, KFError  # noqa: E402
from tests.gpu_cases import oracle_and_gpu, observed_data, tiny_inputs, to_dev  # noqa: E402


def _problem():
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    return inp, orc, gpu


@pytest.mark.parametrize("outer", ["fgmres", "bicgstab"])
def test_iteration_limit_returns_enoconv_with_best_iterate(outer):
    inp, _, gpu = _problem()
    print(f"[case] maxit=1 Newton step 41x19 K=3 outer={outer}", flush=True)
    d = to_dev(observed_data(inp))
    xi, g1, st = gpu.newton_step(d, rtol=1e-12, maxit=1, pc="exact", outer=outer, update_in_place=False)
    assert not st["converged"]
    assert st["outer_iters"] == 1
    assert 0.0 < st["rel_res"] < 1.0          # one step reduced the residual
    assert bool(torch.isfinite(torch.view_as_real(xi)).all()) and bool(torch.isfinite(g1).all())
    assert float(xi.abs().max()) > 0.0


def test_zero_right_hand_side_gives_zero_step():
    inp, orc, gpu = _problem()
    print("[case] zero data residual 41x19 K=3", flush=True)
    # data of gamma_0 itself, from the same FP64 block solve the step makes: the data
    # residual, hence b (b_s = 0 with the regularisation on the update), is exactly zero
    u, _ = gpu.helmholtz_solve(gpu.sources())
    riz = torch.as_tensor(inp["rec_iz"]).long().cuda()
    rix = torch.as_tensor(inp["rec_ix"]).long().cuda()
    d = u[:, riz, rix].contiguous()
    g0 = gpu.get_gamma().clone()
    xi, g1, st = gpu.newton_step(d, rtol=1e-8, maxit=50, pc="exact", update_in_place=False)
    assert st["converged"] and st["outer_iters"] == 0
    assert float(xi.abs().max()) == 0.0
    assert torch.equal(g1, g0)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_non_finite_data_is_reported(bad):
    inp, _, gpu = _problem()
    print(f"[case] {bad} in d, 41x19 K=3", flush=True)
    d = observed_data(inp)
    d[1, 2] = bad
    with pytest.raises(KFError) as e:
        gpu.newton_step(to_dev(d), rtol=1e-8, maxit=50, pc="exact", update_in_place=False)
    assert e.value.status == KF_ENAN
