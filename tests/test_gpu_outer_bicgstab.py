"""The Newton-step KKT system solved by right-preconditioned BiCGStab (the outer solver
the Conclusions propose to halve the memory of GMRES) against the exact step."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_cases import oracle_and_gpu, observed_data, eps_rule, rel, tiny_inputs, to_dev, to_np  # noqa: E402


@pytest.mark.parametrize("pc", ["exact", "inexact"])
def test_bicgstab_outer_step_matches_exact_step(pc):
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3, weights="random")
    print(f"[case] outer BiCGStab 41x19 K=3 pc={pc}", flush=True)
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0, reg_on_update=True)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc, gpu = oracle_and_gpu(inp, eps=eps, reg_on_update=True)
    xi_ref = orc.kkt_solve_schur(u_n, orc.residual(d, u_n))
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-10, maxit=400, pc=pc, outer="bicgstab", update_in_place=False)
    assert st["converged"] and st["rel_res"] <= 1e-10
    xi = to_np(xi)
    for a, b in zip(orc.unpack(xi), orc.unpack(xi_ref)):
        assert rel(a, b) <= 1e-8
    assert rel(to_np(g1), orc.update(orc.unpack(xi_ref)[1])) <= 1e-10
    _, _, stg = gpu.newton_step(to_dev(d), rtol=1e-10, maxit=400, pc=pc, update_in_place=False)
    print(f"BiCGStab {st['outer_iters']} iterations (2 preconditioner applications each), "
          f"FGMRES {stg['outer_iters']}")
