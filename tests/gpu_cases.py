"""Helpers that build the same seeded problem for the oracle and the GPU path."""

import numpy as np
import torch

from oracle.kkt import Problem
from synthetic.configs import make_problem_inputs
from tests.oracle_cases import tiny_inputs


def oracle_and_gpu(inp, gamma=None, eps=None, reg_on_update=True, K=None):
    from paper_2204_06489_amd.solver import KKTProblem
    g = inp["gamma0"] if gamma is None else gamma
    K = inp["K"] if K is None else K
    eps = inp["eps"] if eps is None else eps
    orc = Problem.from_inputs(inp, gamma=g, eps=eps, K=K, reg_on_update=reg_on_update)
    gpu = KKTProblem.from_inputs(inp, gamma=g, eps=eps, K=K, reg_on_update=reg_on_update)
    return orc, gpu


def observed_data(inp, K=None):
    """d = Q u(gamma_true) computed by the oracle."""
    p = Problem.from_inputs(inp, gamma=inp["gamma_true"], eps=1.0, K=K)
    return p.sample(p.forward())


def eps_rule(orc, u_n, rel=1e-2):
    J = orc.jacobians(u_n)
    GN = sum((orc.w[k][:, None] * J[k]).conj().T @ (orc.w[k][:, None] * J[k]) for k in range(orc.K))
    return rel * np.linalg.eigvalsh(GN).max()


def to_dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


__all__ = ["oracle_and_gpu", "observed_data", "eps_rule", "to_dev", "to_np", "rel", "tiny_inputs",
           "make_problem_inputs"]
