"""GPU tests of the torch.autograd.Function around the batched Helmholtz solve.

Forward: u = A(gamma)^-1 f (block factorisation + sweeps).  Backward: mu = A^-H grad_u
and grad_gamma = omega^2 sum_k Re(conj(mu_k) X Z u_k) (the reduced gradient of Section 3
extended to the PML nodes through dA/dgamma = -omega^2 X Z).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle.kkt import Problem, adjoint_gradient_full  # noqa: E402
from paper_2204_06489_amd.autograd import HelmholtzSolve  # noqa: E402
from paper_2204_06489_amd.solver import KKTProblem  # noqa: E402
from synthetic.configs import make_problem_inputs  # noqa: E402
from tests.gpu_cases import observed_data, rel, to_np  # noqa: E402
from tests.oracle_cases import tiny_inputs  # noqa: E402


def _misfit(u, d, rec_iz, rec_ix, w):
    r = d - u[:, rec_iz, rec_ix]
    return 0.5 * torch.sum(torch.abs(w * r) ** 2)


def test_gradient_matches_oracle_and_finite_differences_c0():
    """c0 geometry (101x51, 8 sources, 5 Hz): backward vs the oracle's adjoint gradient
    (1e-10) and vs central differences of the misfit in 20 seeded directions (step 1e-6
    relative to max gamma), |fd - g.dg| <= 1e-6 |g| |dg|."""
    inp = make_problem_inputs("c0")
    print("[case] c0 autograd", flush=True)
    d = torch.as_tensor(observed_data(inp)).cuda()
    gpu = KKTProblem.from_inputs(inp, eps=1.0)
    rec_iz = torch.as_tensor(inp["rec_iz"]).long().cuda()
    rec_ix = torch.as_tensor(inp["rec_ix"]).long().cuda()
    w = torch.as_tensor(inp["w"]).cuda()
    g0 = torch.as_tensor(inp["gamma0"]).cuda().requires_grad_(True)
    u = HelmholtzSolve.apply(g0, gpu, "c128")
    loss = _misfit(u, d, rec_iz, rec_ix, w)
    loss.backward()
    grad = to_np(g0.grad)
    # oracle: grad_u of the misfit is -Q^T W^2 (d - Q u)
    orc = Problem.from_inputs(inp, eps=1.0)
    u_o = orc.forward()
    gu = np.zeros_like(u_o)
    rr = np.asarray(d.cpu()) - orc.sample(u_o)
    gu[:, inp["rec_iz"], inp["rec_ix"]] = -(inp["w"] ** 2) * rr
    ref = adjoint_gradient_full(orc.lu, orc.nx, orc.nz, orc.h, orc.npml, orc.omega, u_o, gu, orc.r0, orc.cref)
    assert rel(grad, ref) <= 1e-10
    # core part equals the oracle's reduced gradient (Section 3)
    assert rel(grad[orc.core], orc.reduced_gradient(u_o, rr)) <= 1e-10
    rng = np.random.default_rng(2)
    gmax = float(np.abs(inp["gamma0"]).max())
    with torch.no_grad():
        for _ in range(20):
            dg = rng.standard_normal(g0.shape)
            t = 1e-6 * gmax / np.abs(dg).max()
            dgt = torch.as_tensor(dg).cuda()
            lp = _misfit(HelmholtzSolve.apply(g0 + t * dgt, gpu, "c128"), d, rec_iz, rec_ix, w).item()
            lm = _misfit(HelmholtzSolve.apply(g0 - t * dgt, gpu, "c128"), d, rec_iz, rec_ix, w).item()
            fd = (lp - lm) / (2 * t)
            assert abs(fd - np.sum(grad * dg)) <= 1e-6 * np.linalg.norm(grad) * np.linalg.norm(dg)


def test_gradcheck_tiny():
    inp = tiny_inputs(nx=13, nz=11, npml=3, K=2)
    gpu = KKTProblem.from_inputs(inp, eps=1.0)
    g0 = torch.as_tensor(inp["gamma0"]).cuda()
    scale = float(g0.abs().max())
    # gradcheck in units of the squared-slowness scale keeps its perturbation meaningful
    x = (g0 / scale).clone().requires_grad_(True)

    def f(xx):
        return HelmholtzSolve.apply(xx * scale, gpu, "c128") * 1e-3

    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_complex64_gradient_error_is_reported():
    """complex64 forward and backward: error against the oracle, stated (FP32 rounding)."""
    inp = tiny_inputs(nx=45, nz=21, npml=5, K=3, weights="random")
    gpu = KKTProblem.from_inputs(inp, eps=1.0)
    g0 = torch.as_tensor(inp["gamma0"]).cuda().requires_grad_(True)
    u = HelmholtzSolve.apply(g0, gpu, "c64")
    c = torch.randn(u.shape, dtype=torch.complex64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    loss = torch.sum(torch.real(torch.conj(c) * u))
    loss.backward()
    orc = Problem.from_inputs(inp, eps=1.0)
    u_o = orc.forward()
    ref = adjoint_gradient_full(orc.lu, orc.nx, orc.nz, orc.h, orc.npml, orc.omega, u_o,
                                c.cpu().numpy().astype(np.complex128), orc.r0, orc.cref)
    err = rel(to_np(g0.grad), ref)
    print(f"complex64 gradient relative error vs FP64 oracle: {err:.2e}")
    assert err <= 1e-3
