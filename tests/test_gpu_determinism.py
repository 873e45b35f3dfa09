"""Run-to-run determinism: every reduction has a fixed order (fixed grids, fixed
partial-sum trees, no floating-point atomics), so repeating a call on the same inputs
gives bitwise the same output: the KKT operator, both preconditioners, the block
solves in every precision and a whole Newton step (its Krylov history included)."""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_cases import oracle_and_gpu, observed_data, eps_rule, tiny_inputs, to_dev  # noqa: E402

SHAPE = dict(nx=81, nz=37, npml=6, K=11, weights="random")


@pytest.fixture(scope="module")
def case():
    inp = tiny_inputs(**SHAPE)
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0)
    u_n = orc.forward()
    _, gpu = oracle_and_gpu(inp, eps=eps_rule(orc, u_n))
    gpu.set_solver_shape(6, 2)
    return gpu, to_dev(d)


def _same(a, b):
    torch.cuda.synchronize()
    return torch.equal(torch.view_as_real(a) if a.is_complex() else a, torch.view_as_real(b) if b.is_complex() else b)


def test_operator_preconditioners_and_solves_repeat_bitwise(case):
    gpu, _ = case
    print("[case] determinism of kkt_apply, precond_apply, helmholtz_solve 81x37 K=11", flush=True)
    g = torch.Generator(device="cuda").manual_seed(7)
    xi = torch.randn(gpu.Nxi, dtype=torch.complex128, device="cuda", generator=g)
    f = gpu.sources()
    u, _ = gpu.helmholtz_solve(f)
    gpu.set_background(u)
    assert _same(gpu.kkt_apply(xi), gpu.kkt_apply(xi))
    for pc in ("exact", "inexact"):
        assert _same(gpu.precond_apply(xi, pc=pc), gpu.precond_apply(xi, pc=pc)), pc
    for prec in ("c128", "c64"):
        ff = f if prec == "c128" else f.to(torch.complex64)
        for adj in (False, True):
            a, _ = gpu.helmholtz_solve(ff, adjoint=adj, prec=prec)
            b, _ = gpu.helmholtz_solve(ff, adjoint=adj, prec=prec)
            assert _same(a, b), (prec, adj)


@pytest.mark.parametrize("pc,fwd", [("exact", "c128"), ("inexact", "mixed")])
def test_newton_step_repeats_bitwise(case, pc, fwd):
    gpu, d = case
    print(f"[case] determinism of newton_step 81x37 K=11 pc={pc} fwd={fwd}", flush=True)
    g0 = gpu.get_gamma().clone()
    runs = []
    for _ in range(2):
        gpu.set_gamma(g0)
        xi, g1, st = gpu.newton_step(d, rtol=1e-8, maxit=300, pc=pc, fwd_prec=fwd, update_in_place=False)
        runs.append((xi.clone(), g1.clone(), st))
    (x0, g0a, s0), (x1, g1a, s1) = runs
    assert _same(x0, x1) and _same(g0a, g1a)
    assert s0["outer_iters"] == s1["outer_iters"] and s0["rel_res_hist"] == s1["rel_res_hist"]
    assert s0["misfit_before"] == s1["misfit_before"]
