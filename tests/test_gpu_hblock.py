"""The L-BFGS H-block in the preconditioner's middle stage (Section 5: approximations of
the reduced Hessian in place of L) against the oracle's two-loop recursion, and Newton
steps that build their own pairs against the exact steps."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from synthetic import complex_normal  # noqa: E402
from tests.gpu_cases import oracle_and_gpu, observed_data, eps_rule, rel, tiny_inputs, to_dev, to_np  # noqa: E402


def _case():
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3, weights="random")
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0, reg_on_update=True)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc, gpu = oracle_and_gpu(inp, eps=eps, reg_on_update=True)
    return orc, gpu, d, u_n


def test_lbfgs_preconditioner_matches_oracle():
    orc, gpu, d, u_n = _case()
    print("[case] L-BFGS H-block 41x19 K=3", flush=True)
    gpu.set_background(to_dev(u_n))
    gpu.set_hblock("lbfgs", max_pairs=2)
    pairs = []
    for k in range(3):                     # three pairs into a ring of two: the oldest drops
        s = complex_normal(orc.Ng, seed=40 + k)
        y = orc.hessian_apply(u_n, s)
        pairs.append((s, y))
        gpu.hblock_add_pair(to_dev(s), to_dev(y))
    yv = complex_normal(orc.nxi, seed=50)
    z = to_np(gpu.precond_apply(to_dev(yv), pc="exact"))
    ref = orc.precond_apply_hblock(u_n, yv, pairs[-2:])
    for a, b in zip(orc.unpack(z), orc.unpack(ref)):
        assert rel(a, b) <= 1e-10
    gpu.set_hblock("eps")
    z0 = to_np(gpu.precond_apply(to_dev(yv), pc="exact"))
    assert rel(z0, orc.precond_apply(u_n, yv)) <= 1e-10


def test_newton_steps_with_lbfgs_hblock_match_exact_steps():
    orc, gpu, d, u_n = _case()
    gpu.set_hblock("lbfgs", max_pairs=4)
    dd = to_dev(d)
    p = orc
    its = []
    for step in range(3):
        xi, g1, st = gpu.newton_step(dd, rtol=1e-11, maxit=300, pc="exact", update_in_place=True)
        assert st["converged"]
        u = p.forward()
        ds_ref = p.unpack(p.kkt_solve_schur(u, p.residual(d, u)))[1]
        assert rel(p.unpack(to_np(xi))[1], ds_ref) <= 1e-9
        p = p.with_gamma(p.update(ds_ref))
        assert rel(to_np(g1), p.gamma) <= 1e-10
        its.append(st["outer_iters"])
    print("FGMRES iterations per step with the L-BFGS H-block:", its)
