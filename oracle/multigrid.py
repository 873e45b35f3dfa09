"""Shifted-Laplacian multigrid as the inexact Helmholtz block solver (oracle; test
infrastructure only).

Section 5 allows any approximation A~ of A in the inexact block-triangular
preconditioner (eq. precond_approx) and names the shifted-Laplacian preconditioner,
inverted approximately by multigrid, as the better choice for realistic problems (the
closing paragraph of Section 5 and the Conclusions).  The paper gives no details; this
oracle takes the common construction, and the GPU path follows the same readings:

* the shifted operator M = A(gamma (1 + i beta)) (beta = 0.5): the mass term
  -omega^2 gamma X Z is multiplied by 1 + i beta, which moves the spectrum into the same
  (lower) half-plane as the PML damping under the e^{-i w t} convention;
* levels by standard coarsening of the vertex grid (n -> (n + 1) / 2 while both sizes
  are odd and the smaller one is at least `n_min`), spacing doubled, PML width halved
  (npml // 2 cells, the same profile law), gamma injected (every second node);
  every level's operator is the shifted 5-point PML operator rediscretised on its grid;
* smoothing by line Jacobi: a z-line sweep (every grid column solved exactly for its own
  unknowns, the x-neighbours taken from the previous iterate) then an x-line sweep
  (every row) before the coarse correction, the reverse order after it; lines absorb
  the strong coupling across the PML strips, where the stretch factors make the
  operator anisotropic;
* full-weighting restriction R = P^T / 4 and bilinear prolongation P;
* the coarsest level solved exactly (banded LU);
* the outer iteration is BiCGStab (van der Vorst) on A, right-preconditioned by one
  V-cycle, stopped at ||b - A x|| <= rtol ||b|| per right-hand side.

A^H solves use A^H = conj(A) (A is complex symmetric): x = conj(solve(conj(b))).
"""

import numpy as np
import scipy.sparse as sp
from scipy.linalg import solve_banded

from .helmholtz import assemble_A, BandedLU
from .pml import stretch


def shifted_operator(nx, nz, h, npml, omega, gamma, r0, cref, beta):
    """A(gamma (1 + i beta)) as CSR: A minus i beta omega^2 diag(gamma X Z)."""
    A = assemble_A(nx, nz, h, npml, omega, gamma, r0, cref)
    Xn, _ = stretch(nx, h, npml, omega, r0, cref)
    Zn, _ = stretch(nz, h, npml, omega, r0, cref)
    mass = omega ** 2 * np.asarray(gamma) * (Zn[:, None] * Xn[None, :])
    return (A - sp.diags(1j * beta * mass.ravel())).tocsr()


def prolongation_1d(nc):
    """Linear interpolation from nc coarse nodes to 2 nc - 1 fine nodes."""
    n = 2 * nc - 1
    rows, cols, vals = [], [], []
    for I in range(nc):
        rows.append(2 * I); cols.append(I); vals.append(1.0)
        if I + 1 < nc:
            rows += [2 * I + 1, 2 * I + 1]; cols += [I, I + 1]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


class Level:
    def __init__(self, nx, nz, h, npml, gamma, M):
        self.nx, self.nz, self.h, self.npml, self.gamma, self.M = nx, nz, h, npml, gamma, M
        self.P = None        # prolongation from the next level
        self.lu = None       # coarsest level only


def build_levels(nx, nz, h, npml, omega, gamma, r0, cref, beta=0.5, n_min=20, max_levels=8):
    """The multigrid hierarchy of the shifted operator (see the module docstring)."""
    levels = []
    g = np.asarray(gamma, dtype=np.float64)
    while True:
        lev = Level(nx, nz, h, npml, g, shifted_operator(nx, nz, h, npml, omega, g, r0, cref, beta))
        levels.append(lev)
        if nx % 2 == 0 or nz % 2 == 0 or min(nx, nz) < n_min or len(levels) == max_levels:
            break
        ncx, ncz = (nx + 1) // 2, (nz + 1) // 2
        lev.P = sp.kron(prolongation_1d(ncz), prolongation_1d(ncx)).tocsr()
        nx, nz, h, npml = ncx, ncz, 2.0 * h, npml // 2
        g = g[::2, ::2].copy()
    levels[-1].lu = BandedLU(levels[-1].M, levels[-1].nx, levels[-1].nz)
    return levels


def line_jacobi(lev, x, b, direction):
    """One line-Jacobi sweep: every z-line (direction 'z', one per grid column) or x-line
    (one per row) solves its tridiagonal part of M exactly, the other couplings taken
    from x.  x, b: [nz][nx]."""
    M = lev.M
    nx, nz = lev.nx, lev.nz
    r = b.ravel() - M @ x.ravel()          # residual with every coupling
    out = x.copy()
    if direction == "z":
        for i in range(nx):
            idx = np.arange(nz) * nx + i
            T = M[idx][:, idx].toarray()
            ab = np.zeros((3, nz), np.complex128)
            ab[0, 1:] = np.diag(T, 1)
            ab[1] = np.diag(T)
            ab[2, :-1] = np.diag(T, -1)
            out[:, i] = x[:, i] + solve_banded((1, 1), ab, r[idx])
    else:
        for j in range(nz):
            idx = j * nx + np.arange(nx)
            T = M[idx][:, idx].toarray()
            ab = np.zeros((3, nx), np.complex128)
            ab[0, 1:] = np.diag(T, 1)
            ab[1] = np.diag(T)
            ab[2, :-1] = np.diag(T, -1)
            out[j, :] = x[j, :] + solve_banded((1, 1), ab, r[idx])
    return out


def vcycle(levels, b, level=0):
    """x ~= M^-1 b by one V-cycle from `level` down (b: [nz][nx] of that level)."""
    lev = levels[level]
    if lev.lu is not None:
        return lev.lu.solve(b)
    x = np.zeros_like(b)
    x = line_jacobi(lev, x, b, "z")
    x = line_jacobi(lev, x, b, "x")
    r = b.ravel() - lev.M @ x.ravel()
    nxt = levels[level + 1]
    rc = (lev.P.T @ r / 4.0).reshape(nxt.nz, nxt.nx)
    ec = vcycle(levels, rc, level + 1)
    x = x + (lev.P @ ec.ravel()).reshape(lev.nz, lev.nx)
    x = line_jacobi(lev, x, b, "x")
    x = line_jacobi(lev, x, b, "z")
    return x


def bicgstab(A, precond, b, rtol=1e-3, maxit=500):
    """BiCGStab (van der Vorst) for A x = b from x = 0, right-preconditioned: the
    search directions are preconditioned and ||b - A x|| <= rtol ||b|| stops it.
    Returns (x, history of ||b - A x|| / ||b||)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    if nb == 0.0:
        return x, hist
    r = b.copy()
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for _ in range(maxit):
        rho_new = np.vdot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = precond(p)
        v = A @ ph
        alpha = rho_new / np.vdot(rhat, v)
        s = r - alpha * v
        sh = precond(s)
        t = A @ sh
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho = rho_new
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
    return x, hist


class MultigridSolver:
    """A x = b (or A^H x = b) for every source by BiCGStab with one V-cycle of the
    shifted operator per preconditioning step."""

    def __init__(self, nx, nz, h, npml, omega, gamma, r0, cref, beta=0.5, n_min=20):
        self.nx, self.nz = nx, nz
        self.A = assemble_A(nx, nz, h, npml, omega, gamma, r0, cref)
        self.levels = build_levels(nx, nz, h, npml, omega, gamma, r0, cref, beta, n_min)

    def precond(self, v):
        return vcycle(self.levels, np.asarray(v).reshape(self.nz, self.nx)).ravel()

    def solve(self, b, adjoint=False, rtol=1e-3, maxit=500):
        """x[k] for every b[k] ([K][nz][nx]); returns (x, iterations per source)."""
        b = np.asarray(b, dtype=np.complex128)
        x = np.empty_like(b)
        its = []
        for k in range(b.shape[0]):
            rhs = np.conj(b[k]) if adjoint else b[k]
            xk, hist = bicgstab(self.A, self.precond, rhs.ravel(), rtol, maxit)
            x[k] = (np.conj(xk) if adjoint else xk).reshape(self.nz, self.nx)
            its.append(len(hist) - 1)
        return x, its
