"""The shifted-Laplacian multigrid block solver (the inexact A~ of the third
preconditioner variant, Section 5) against the oracle's multigrid: one V-cycle element
by element (the same levels, smoother, transfers and exact coarsest solve), the
BiCGStab solves against their tolerance and the oracle's iteration counts, the
preconditioner's stage bounds, and a Newton step with it against the exact step."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle.multigrid import MultigridSolver, build_levels, vcycle  # noqa: E402
from synthetic import complex_normal  # noqa: E402
from tests.gpu_cases import (oracle_and_gpu, observed_data, eps_rule, make_problem_inputs, rel, tiny_inputs,  # noqa: E402
                             to_dev, to_np)

SHAPES = [dict(nx=81, nz=37, npml=5, K=3), dict(nx=65, nz=45, npml=4, K=5)]


def _levels(inp, n_min):
    return build_levels(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"], inp["pml_r0"],
                        inp["pml_cref"], 0.5, n_min)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_vcycle_matches_oracle(shape, prec, tol):
    inp = tiny_inputs(**shape)
    print(f"[case] V-cycle {shape} {prec}", flush=True)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    gpu.set_multigrid(prec=prec, n_min=8)
    levels = _levels(inp, 8)
    b = complex_normal(gpu.field_shape, seed=12)
    x = to_np(gpu.mg_vcycle(to_dev(b)))
    dims = gpu.mg_levels()
    assert dims == [(lv.nx, lv.nz) for lv in levels] and len(dims) >= 3, dims
    for k in range(gpu.K):
        ref = vcycle(levels, b[k])
        assert rel(x[k], ref) <= tol, (k, rel(x[k], ref))


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_multigrid_solve_meets_tolerance(adjoint, prec):
    inp = make_problem_inputs("c0", 0)
    print(f"[case] MG solve c0 adjoint={adjoint} {prec}", flush=True)
    orc, gpu = oracle_and_gpu(inp, eps=1.0, K=3)
    gpu.set_multigrid(prec=prec)
    b = complex_normal(gpu.field_shape, seed=13)
    x, st = gpu.helmholtz_solve_mg(to_dev(b), adjoint=adjoint, rtol=1e-3, maxit=100)
    assert st["converged"] and st["rel_res_max"] <= 1.5e-3, st
    ms = MultigridSolver(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"], inp["pml_r0"],
                         inp["pml_cref"])
    xo, its = ms.solve(b, adjoint=adjoint, rtol=1e-3)
    print(f"GPU {st['iters']} iterations ({st['levels']} levels), oracle {its}; true residual {st['rel_res_max']:.2e}")
    assert abs(st["iters"] - max(its)) <= (1 if prec == "c128" else 3)
    # tighter: the solve converges on toward the exact solution
    x2, st2 = gpu.helmholtz_solve_mg(to_dev(b), adjoint=adjoint, rtol=1e-8 if prec == "c128" else 1e-5, maxit=300)
    ref = orc.lu.solve(b, adjoint=adjoint)
    assert st2["converged"] and rel(to_np(x2), ref) <= (1e-6 if prec == "c128" else 1e-3)


def test_multigrid_preconditioner_stage_bounds():
    """The variant's preconditioner (eq. precond_approx with multigrid block solves): each
    block solve within the inner tolerance, the middle stage exactly the stage-2 formula."""
    inp = tiny_inputs(nx=81, nz=37, npml=5, K=3, nrec=9)
    orc, gpu = oracle_and_gpu(inp, eps=2.3e9)
    gpu.set_multigrid(prec="c64", inner_rtol=1e-3, n_min=8)
    u_n = orc.forward()
    gpu.set_background(to_dev(u_n))
    y = complex_normal(orc.nxi, seed=14)
    z = to_np(gpu.precond_apply(to_dev(y), pc="multigrid"))
    yu, ys, yl = orc.unpack(y)
    zu, zs, zl = orc.unpack(z)
    AH = orc.A.conj().T
    for k in range(orc.K):
        assert np.linalg.norm(AH @ zl[k].ravel() - yu[k].ravel()) <= 1.5e-3 * np.linalg.norm(yu[k])
    w2 = orc.omega ** 2
    zs_ref = (ys + w2 * np.sum(np.conj(u_n) * zl, axis=0).ravel()[orc.core_idx]) / orc.eps
    assert rel(zs, zs_ref) <= 1e-12
    ext = np.zeros(orc.Nu, complex)
    ext[orc.core_idx] = zs
    rhs = yl + w2 * u_n * ext.reshape(orc.nz, orc.nx)[None]
    for k in range(orc.K):
        assert np.linalg.norm(orc.A @ zu[k].ravel() - rhs[k].ravel()) <= 1.5e-3 * np.linalg.norm(rhs[k])


def test_newton_step_with_multigrid_preconditioner():
    inp = tiny_inputs(nx=81, nz=37, npml=5, K=3, weights="random")
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0, reg_on_update=True)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc, gpu = oracle_and_gpu(inp, eps=eps, reg_on_update=True)
    gpu.set_multigrid(prec="c64", inner_rtol=1e-3, n_min=8)
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-9, restart=30, maxit=300, pc="multigrid", update_in_place=False)
    assert st["converged"] and st["rel_res"] <= 1e-9
    ref = orc.unpack(orc.kkt_solve_schur(u_n, orc.residual(d, u_n)))[1]
    print(f"multigrid-preconditioned step: {st['outer_iters']} iterations, ds error {rel(orc.unpack(to_np(xi))[1], ref):.1e}")
    assert rel(orc.unpack(to_np(xi))[1], ref) <= 1e-6
