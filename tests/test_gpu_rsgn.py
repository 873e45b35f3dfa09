"""Reduced-space Gauss-Newton by CG on the GPU (rsgn_cg_step, Section 3; Table 1 "CG")
against the oracle: the normal-equation solution by dense Cholesky (pinned by numpy's
least squares), the oracle's own CG iteration count, and the real-constrained step
against the real least-squares minimiser."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_cases import oracle_and_gpu, observed_data, eps_rule, to_dev, to_np, rel, tiny_inputs  # noqa: E402


def _setup(reg_on_update, **kw):
    inp = tiny_inputs(weights="random", **kw)
    print(f"[case] rsgn {kw} reg_on_update={reg_on_update}", flush=True)
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0, reg_on_update=reg_on_update)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc, gpu = oracle_and_gpu(inp, eps=eps, reg_on_update=reg_on_update)
    return orc, gpu, d, u_n


@pytest.mark.parametrize("reg", [False, True])
@pytest.mark.parametrize("shape", [dict(nx=41, nz=19, npml=4, K=3), dict(nx=67, nz=37, npml=5, K=5, nrec=9)])
def test_rsgn_step_matches_normal_equations(reg, shape):
    orc, gpu, d, u_n = _setup(reg, **shape)
    r = orc.residual(d, u_n)
    H, g = orc.normal_system(u_n, r)
    ref = np.linalg.solve(H, g)
    ds, g1, st = gpu.rsgn_step(to_dev(d), rtol=1e-12, maxit=500, update_in_place=False)
    assert st["converged"] and st["true_rel_res"] <= 1e-11
    assert rel(to_np(ds), ref) <= 1e-10
    assert rel(to_np(g1), orc.update(ref)) <= 1e-12
    _, hist = orc.rsgn_cg(u_n, r, tol=1e-12, maxit=500)
    print(f"GPU CG {st['iters']} iterations ({st['solves']} batched solves), oracle CG {len(hist) - 1}")
    assert abs(st["iters"] - (len(hist) - 1)) <= 2
    # complex64 factors inside FP64 refinement for every block solve
    dsm, _, stm = gpu.rsgn_step(to_dev(d), rtol=1e-10, maxit=500, solve_prec="mixed", solve_rtol=1e-12,
                                fwd_prec="mixed", fwd_rtol=1e-12, update_in_place=False)
    assert stm["converged"] and rel(to_np(dsm), ref) <= 1e-8


def test_real_constrained_rsgn_step():
    orc, gpu, d, u_n = _setup(True, nx=41, nz=19, npml=4, K=3)
    r = orc.residual(d, u_n)
    Hr, gr = orc.normal_system_real(u_n, r)
    ref = np.linalg.solve(Hr, gr)
    ds, _, st = gpu.rsgn_step(to_dev(d), rtol=1e-12, maxit=500, real_constrained=True, update_in_place=False)
    ds = to_np(ds)
    assert st["converged"] and np.abs(ds.imag).max() == 0.0
    assert rel(ds.real, ref) <= 1e-10


def test_rsgn_step_updates_gamma_in_place_and_reduces_misfit():
    orc, gpu, d, u_n = _setup(True, nx=41, nz=19, npml=4, K=3)
    dd = to_dev(d)
    _, g1, st0 = gpu.rsgn_step(dd, rtol=1e-8, update_in_place=True)
    assert torch.equal(gpu.get_gamma(), g1)
    _, _, st1 = gpu.rsgn_step(dd, rtol=1e-8, update_in_place=True)
    assert st1["misfit_before"] < st0["misfit_before"]
