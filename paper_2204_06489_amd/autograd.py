"""torch.autograd.Function for the batched Helmholtz solve u = A(gamma)^-1 f.

Forward: the block factorisation of A(gamma) and the batched forward sweep.
Backward: the hand-written adjoint solve mu = A^-H grad_u and the kernel
grad_gamma = omega^2 sum_k Re(conj(mu_k) X Z u_k) (the reduced gradient of
Section 3; X = Z = 1 on the core).  Both run in libkktfwi.so.
"""

import torch

from .solver import KKTProblem


class HelmholtzSolve(torch.autograd.Function):
    """u = HelmholtzSolve.apply(gamma, problem, prec) with prec in {"c128", "c64"}.

    ``gamma`` is the real [nz][nx] squared slowness (float64, on the GPU); the
    sources are the problem's unit point sources.  The returned u is
    complex128 (c128) or complex64 (c64), [K][nz][nx]."""

    @staticmethod
    def forward(ctx, gamma, problem: KKTProblem, prec="c128"):
        problem.set_gamma(gamma.detach())
        f = problem.sources()
        if prec == "c64":
            f = f.to(torch.complex64)
        u, _ = problem.helmholtz_solve(f, adjoint=False, prec=prec)
        ctx.problem, ctx.prec = problem, prec
        ctx.token = problem.gamma_token
        ctx.save_for_backward(gamma, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        gamma, u = ctx.saved_tensors
        problem, prec = ctx.problem, ctx.prec
        # the factors belong to another gamma if the problem was reused in between
        if problem.gamma_token != ctx.token:
            problem.set_gamma(gamma.detach())
        dt = torch.complex64 if prec == "c64" else torch.complex128
        g = problem.adjoint_gradient(u.contiguous(), grad_u.to(dt).contiguous(), prec=prec)
        return g.to(gamma.dtype), None, None


def helmholtz_solve(gamma, problem, prec="c128"):
    return HelmholtzSolve.apply(gamma, problem, prec)
