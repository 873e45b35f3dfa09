"""Pins of the oracle functions that produce inputs or judge results: the Gauss-Newton
operator and its largest eigenvalue (which fix eps for every workload), the point
sources, and the KKT first-order-condition residuals.

Each pin ties the function to something other than itself (the finite-difference-
pinned Jacobian, a dense eigensolver, the Hankel Green's function, residuals known
by construction), and a mutation check plants a plausible mistake in a copy of the
oracle function and shows that the same pin rejects it.
"""

import json

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.special import hankel1

from oracle.kkt import Problem
from oracle.make_eps import lambda_max, REL
from synthetic.configs import EPS_TABLE_PATH, make_problem_inputs
from tests.oracle_cases import tiny_inputs


def _prob(weights="random", **kw):
    inp = tiny_inputs(weights=weights, **kw)
    p = Problem.from_inputs(inp, eps=1.0)
    return p, p.forward()


def _gn_from_jacobians(p, u_n):
    """sum_k J_k^* W_k^2 J_k as a dense matrix, from the FD-pinned Jacobians."""
    J = p.jacobians(u_n)
    return sum((p.w[k][:, None] * J[k]).conj().T @ (p.w[k][:, None] * J[k]) for k in range(p.K))


def _gn_operator_pin(p, u_n, apply):
    GN = _gn_from_jacobians(p, u_n)
    rng = np.random.default_rng(21)
    for _ in range(3):
        v = rng.standard_normal(p.Ng) + 1j * rng.standard_normal(p.Ng)
        ref = GN @ v
        if np.linalg.norm(apply(v) - ref) > 1e-11 * np.linalg.norm(ref):
            return False
    return True


def test_gn_operator_equals_jacobian_normal_matrix():
    """gn_operator(v) = sum_k J_k^* W_k^2 J_k v (Section 3, Hessian without L) with random
    receiver weights, J pinned by finite differences of the forward map elsewhere."""
    p, u_n = _prob()
    assert _gn_operator_pin(p, u_n, p.gn_operator(u_n))


def test_gn_operator_pin_rejects_planted_mistakes():
    """The same pin fails for W^2 dropped, W instead of W^2, and omega^2 applied once."""
    p, u_n = _prob()
    Qd = p.Q().toarray().reshape(p.nrec, p.nz, p.nx).astype(np.complex128)
    Gc = p.lu.solve(Qd, adjoint=True).reshape(p.nrec, -1)[:, p.core_idx]
    uc = np.asarray(u_n).reshape(p.K, -1)[:, p.core_idx]
    w2 = p.omega ** 2

    def mutant(weight_pow, omega_pow):
        def apply(v):
            out = np.zeros(p.Ng, np.complex128)
            for k in range(p.K):
                y = w2 * (np.conj(Gc) @ (uc[k] * v))
                out += p.omega ** omega_pow * np.conj(uc[k]) * (Gc.T @ (p.w[k] ** weight_pow * y))
            return out
        return apply
    assert _gn_operator_pin(p, u_n, mutant(2, 2))          # the correct form passes
    assert not _gn_operator_pin(p, u_n, mutant(0, 2))      # W^2 dropped
    assert not _gn_operator_pin(p, u_n, mutant(1, 2))      # W instead of W^2
    assert not _gn_operator_pin(p, u_n, mutant(2, 0))      # omega^2 only once


def test_lambda_max_matches_dense_eigensolver():
    """Power iteration's Rayleigh quotient never exceeds lambda_max and converges to
    numpy's eigvalsh of the dense Gauss-Newton matrix."""
    p, u_n = _prob(weights="ones")
    ref = np.linalg.eigvalsh(_gn_from_jacobians(p, u_n)).max()
    apply = p.gn_operator(u_n)
    lam20 = lambda_max(apply, p.Ng, 20)
    lam200 = lambda_max(apply, p.Ng, 200)
    assert lam20 <= ref * (1 + 1e-12) and lam200 <= ref * (1 + 1e-12)
    assert abs(lam200 - ref) <= 1e-8 * ref
    assert abs(lam20 - ref) <= 1e-2 * ref


def test_stored_eps_of_the_smallest_workload_matches_eigvalsh():
    """The eps literal of the 101 x 51, 8-source, 5 Hz workload (written by make_eps with 20
    power iterations) is 1e-2 lambda_max of the dense sum_k J_k^* J_k at gamma0."""
    table = json.load(open(EPS_TABLE_PATH))
    inp = make_problem_inputs("c0", 0)
    p = Problem.from_inputs(inp, eps=1.0)
    ref = REL * np.linalg.eigvalsh(_gn_from_jacobians(p, p.forward())).max()
    assert abs(table["c0/g0/5"] - ref) <= 1e-3 * ref
    assert table["c0/g0/5"] <= ref * (1 + 1e-12)


def _hankel_error(ppw, v=2000.0, freq=5.0, src_scale=None):
    """Relative L2 error of Problem.forward()'s point-source field vs (i/4) H0^(1)(k r) on
    the annulus 5h <= r <= one wavelength (PML one wavelength wide, R0 = 1e-6)."""
    lam = v / freq
    h = lam / ppw
    npml = int(round(ppw))
    half_core = int(np.ceil((lam + 10 * h) / h))
    n = 2 * (half_core + npml) + 1
    c = n // 2
    p = Problem(n, n, h, npml, 2 * np.pi * freq, np.full((n, n), 1.0 / v ** 2), [c], [c], [c], [npml],
                eps=1.0, pml_r0=1e-6, pml_cref=v)
    if src_scale is not None:         # a planted mistake in the source normalisation
        p.sources = lambda: Problem.sources(p) * src_scale
    u = p.forward()[0]
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = h * np.hypot(ii - c, jj - c)
    ring = (r >= 5 * h) & (r <= lam)
    exact = 0.25j * hankel1(0, 2 * np.pi * freq / v * r[ring])
    return np.linalg.norm(u[ring] - exact) / np.linalg.norm(exact)


def test_problem_sources_and_forward_give_the_green_function():
    """Problem.sources() (f = e_src / h^2) through Problem.forward() is the free-space
    Green's function (Section 2 source term; e^{-i w t} convention)."""
    assert _hankel_error(60) <= 0.01


def test_green_pin_rejects_source_scaled_by_h_instead_of_h2():
    lam_h = 2000.0 / 5.0 / 60
    assert _hankel_error(60, src_scale=lam_h) > 0.5


def _kkt_setup():
    inp = tiny_inputs(weights="random")
    pt = Problem.from_inputs(inp, gamma=inp["gamma_true"], eps=1.0)
    d = pt.sample(pt.forward())
    p = Problem.from_inputs(inp, eps=1.0, reg_on_update=True)
    u_n = p.forward()
    r = p.residual(d, u_n)
    b = p.rhs(r)
    xi = p.kkt_solve_dense(u_n, b)
    return p, u_n, b, xi


def _denominators(p, u_n, xi, b):
    M = p.assemble_M(u_n)
    mag = p.unpack(abs(M) @ np.abs(xi) + 0j)
    bb = p.unpack(np.asarray(b))
    return [np.linalg.norm(mag[t]) + np.linalg.norm(bb[t]) for t in range(3)]


def test_kkt_rows_of_a_state_perturbation_are_known():
    """xi* + (delta_u, 0, 0) with delta_u zero on the receiver nodes: the first-order
    conditions (Section 4) then fail only in the state row, by exactly A delta_u."""
    p, u_n, b, xi = _kkt_setup()
    rng = np.random.default_rng(8)
    du = rng.standard_normal((p.K, p.nz, p.nx)) + 1j * rng.standard_normal((p.K, p.nz, p.nx))
    du[:, p.rec_iz, p.rec_ix] = 0.0
    du *= 1e-3 * np.abs(xi[:p.K * p.Nu]).max()
    pert = xi + p.pack(du, np.zeros(p.Ng), np.zeros_like(du))
    rows = p.kkt_rows(u_n, pert, b)
    den = _denominators(p, u_n, pert, b)
    expect = np.linalg.norm(np.stack([p.A @ du[k].ravel() for k in range(p.K)])) / den[2]
    assert rows[0] <= 1e-12 and rows[1] <= 1e-12
    assert rows[2] == pytest.approx(expect, rel=1e-8)
    assert rows[2] > 1e-6


def test_kkt_rows_of_a_multiplier_perturbation_are_known():
    """xi* + (0, 0, delta_lambda): the residual is A^* delta_lambda in the state-adjoint row
    and omega^2 E^T sum_k conj(u_k) delta_lambda_k in the control row (P^* delta_lambda)."""
    p, u_n, b, xi = _kkt_setup()
    rng = np.random.default_rng(9)
    dl = rng.standard_normal((p.K, p.nz, p.nx)) + 1j * rng.standard_normal((p.K, p.nz, p.nx))
    dl *= 1e-3 * np.abs(xi[-p.K * p.Nu:]).max()
    pert = xi + p.pack(np.zeros_like(dl), np.zeros(p.Ng), dl)
    rows = p.kkt_rows(u_n, pert, b)
    den = _denominators(p, u_n, pert, b)
    AH = p.A.conj().T
    r1 = np.linalg.norm(np.stack([AH @ dl[k].ravel() for k in range(p.K)]))
    r2 = np.linalg.norm(p.omega ** 2 * np.sum(np.conj(u_n) * dl, axis=0).ravel()[p.core_idx])
    assert rows[0] == pytest.approx(r1 / den[0], rel=1e-8)
    assert rows[1] == pytest.approx(r2 / den[1], rel=1e-8)
    assert rows[2] <= 1e-12
