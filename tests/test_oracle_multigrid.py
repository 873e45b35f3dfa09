"""Pins of the oracle's shifted-Laplacian multigrid (the inexact block solver of
Section 5): transfer operators against exact interpolation of linear functions, the
shifted operator against its no-PML textbook form, the line smoother against a direct
solve where a line is the whole system, V-cycle convergence on the Poisson problem
(the textbook case) and on the shifted Helmholtz operator, and BiCGStab against its
stopping rule and the one-step exact-preconditioner case."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.helmholtz import assemble_A
from oracle.multigrid import (MultigridSolver, bicgstab, build_levels, line_jacobi, prolongation_1d,
                              shifted_operator, vcycle)
from synthetic.configs import make_problem_inputs


def test_prolongation_and_full_weighting_are_exact_on_linear_functions():
    nc = 9
    P = prolongation_1d(nc).toarray()
    xc = np.linspace(0.0, 1.0, nc)
    xf = np.linspace(0.0, 1.0, 2 * nc - 1)
    assert np.allclose(P @ (3 * xc - 1), 3 * xf - 1, atol=1e-15)
    P2 = sp.kron(prolongation_1d(5), prolongation_1d(7))
    zz, xx = np.meshgrid(np.arange(9.0), np.arange(13.0), indexing="ij")
    f = 2.0 * xx - 0.5 * zz + 1.0
    fc = (P2.T @ f.ravel() / 4.0).reshape(5, 7)
    # full weighting reproduces a linear function at interior coarse nodes
    assert np.allclose(fc[1:-1, 1:-1], f[2:-2:2, 2:-2:2], atol=1e-13)


def test_shifted_operator_without_pml_is_laplacian_minus_shifted_mass():
    nx, nz, h, omega, beta = 13, 9, 7.0, 2 * np.pi * 3.0, 0.5
    g = np.random.default_rng(1).uniform(1 / 4000 ** 2, 1 / 1500 ** 2, (nz, nx))
    M = shifted_operator(nx, nz, h, 0, omega, g, 1e-3, 3000.0, beta)
    lap = (sp.kron(sp.identity(nz), sp.diags([-1, 2, -1], [-1, 0, 1], (nx, nx))) +
           sp.kron(sp.diags([-1, 2, -1], [-1, 0, 1], (nz, nz)), sp.identity(nx))) / h ** 2
    ref = lap - (1 + 1j * beta) * omega ** 2 * sp.diags(g.ravel())
    assert abs(M - ref).max() <= 1e-12 * abs(ref).max()
    Mp = shifted_operator(23, 17, 10.0, 5, omega, np.full((17, 23), 1 / 2000 ** 2), 1e-3, 3000.0, beta)
    assert abs(Mp - Mp.T).max() == 0.0          # complex symmetric, like A
    A0 = assemble_A(23, 17, 10.0, 5, omega, np.full((17, 23), 1 / 2000 ** 2), 1e-3, 3000.0)
    assert abs(shifted_operator(23, 17, 10.0, 5, omega, np.full((17, 23), 1 / 2000 ** 2), 1e-3, 3000.0, 0.0)
               - A0).max() == 0.0


@pytest.mark.parametrize("direction", ["z", "x"])
def test_line_jacobi_is_exact_when_a_line_is_the_whole_grid(direction):
    nx, nz = (1, 31) if direction == "z" else (31, 1)
    omega = 2 * np.pi * 4.0
    lev = build_levels(nx, nz, 10.0, 0, omega, np.full((nz, nx), 1 / 2000 ** 2), 1e-3, 3000.0)[0]
    rng = np.random.default_rng(3)
    b = rng.standard_normal((nz, nx)) + 1j * rng.standard_normal((nz, nx))
    x0 = rng.standard_normal((nz, nx)) + 0j
    x = line_jacobi(lev, x0, b, direction)
    ref = spla.spsolve(lev.M.tocsc(), b.ravel()).reshape(nz, nx)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def _vcycle_factor(levels, n_cycles=6, seed=0):
    lev = levels[0]
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((lev.nz, lev.nx)) + 1j * rng.standard_normal((lev.nz, lev.nx))
    x = np.zeros_like(b)
    res = []
    for _ in range(n_cycles):
        x = x + vcycle(levels, b - (lev.M @ x.ravel()).reshape(b.shape))
        res.append(np.linalg.norm(b.ravel() - lev.M @ x.ravel()) / np.linalg.norm(b))
    return (res[-1] / res[1]) ** (1.0 / (n_cycles - 2)), res


def test_two_grid_cycle_converges_grid_independently_on_poisson():
    """omega -> 0 and no PML: the two-grid cycle (line smoothing, full weighting, bilinear
    interpolation, rediscretised coarse operator) contracts the residual of the
    Laplacian by a factor independent of the grid size (about 0.33 here; the coarse grid
    of this vertex layout puts its zero boundary one fine cell further out, which is
    what keeps it above the textbook 0.1 of a nested boundary)."""
    rhos = []
    for n in (33, 65, 129):
        levels = build_levels(n, n, 1.0, 0, 1e-9, np.ones((n, n)), 1e-3, 1.0, n_min=8, max_levels=2)
        rho, _ = _vcycle_factor(levels)
        rhos.append(rho)
    assert max(rhos) < 0.4 and max(rhos) - min(rhos) < 0.05, rhos


def test_vcycle_converges_on_the_shifted_helmholtz_operator():
    inp = make_problem_inputs("c0", 0)
    levels = build_levels(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"],
                          inp["pml_r0"], inp["pml_cref"])
    rho, res = _vcycle_factor(levels)
    assert rho < 0.8 and res[-1] < 0.05, (rho, res)


def test_bicgstab_with_exact_preconditioner_takes_one_iteration():
    inp = make_problem_inputs("c0", 0)
    A = assemble_A(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"],
                   inp["pml_r0"], inp["pml_cref"])
    lu = spla.splu(A.tocsc())
    b = np.random.default_rng(5).standard_normal(A.shape[0]) + 0j
    x, hist = bicgstab(A, lu.solve, b, rtol=1e-10, maxit=5)
    assert len(hist) - 1 == 1 and hist[-1] <= 1e-10


@pytest.mark.parametrize("adjoint", [False, True])
def test_multigrid_solver_meets_its_tolerance(adjoint):
    inp = make_problem_inputs("c0", 0)
    s = MultigridSolver(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"],
                        inp["pml_r0"], inp["pml_cref"])
    rng = np.random.default_rng(6)
    b = rng.standard_normal((2, inp["nz"], inp["nx"])) + 1j * rng.standard_normal((2, inp["nz"], inp["nx"]))
    x, its = s.solve(b, adjoint=adjoint, rtol=1e-3)
    A = s.A.conj().T if adjoint else s.A
    for k in range(2):
        assert np.linalg.norm(b[k].ravel() - A @ x[k].ravel()) <= 1e-3 * np.linalg.norm(b[k])
    assert max(its) <= 30
