"""Discrete Helmholtz operator with PML and its banded LU (oracle; test infrastructure only).

Section 2: the PML form of the Helmholtz equation multiplied through by XZ,

    -Z d/dx (1/X dU/dx) - X d/dz (1/Z dU/dz) - omega^2 gamma X Z U = F,  U = 0 on the boundary,

discretised by finite differences into A u = f (the discrete forward problem).
The paper does not print its stencil; this oracle takes the conservative
5-point scheme with the outer factor at the node and the inner 1/X, 1/Z at the
half-nodes between neighbours.  Grid values outside the listed nodes are zero
(the Dirichlet condition).  Without PML (X = Z = 1) the matrix is the standard
-Laplacian - omega^2 diag(gamma), the special case the paper states.

Unknowns are ordered p = j*nx + i (x fastest), i.e. fields are [nz][nx].
"""

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lapack

from .pml import stretch


def assemble_A(nx, nz, h, npml, omega, gamma, r0=1e-3, cref=4000.0):
    """Sparse CSR matrix A (nx*nz square, complex128) of the PML Helmholtz operator.

    Row (i, j):
      (A u)_ij = -(Z_j/h^2) [ (u_{i+1,j} - u_ij)/X_{i+1/2} - (u_ij - u_{i-1,j})/X_{i-1/2} ]
                 -(X_i/h^2) [ (u_{i,j+1} - u_ij)/Z_{j+1/2} - (u_ij - u_{i,j-1})/Z_{j-1/2} ]
                 - omega^2 gamma_ij X_i Z_j u_ij
    """
    gamma = np.asarray(gamma, dtype=np.float64)
    assert gamma.shape == (nz, nx)
    Xn, Xh = stretch(nx, h, npml, omega, r0, cref)
    Zn, Zh = stretch(nz, h, npml, omega, r0, cref)
    jj, ii = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    p = jj * nx + ii
    h2 = h * h
    # neighbour weights (off-diagonal entries)
    w_xm = -Zn[jj] / (h2 * Xh[ii])          # coupling to (i-1, j) through face i-1/2
    w_xp = -Zn[jj] / (h2 * Xh[ii + 1])      # coupling to (i+1, j) through face i+1/2
    w_zm = -Xn[ii] / (h2 * Zh[jj])          # coupling to (i, j-1) through face j-1/2
    w_zp = -Xn[ii] / (h2 * Zh[jj + 1])      # coupling to (i, j+1) through face j+1/2
    diag = -(w_xm + w_xp + w_zm + w_zp) - omega ** 2 * gamma * Xn[ii] * Zn[jj]

    rows, cols, vals = [p.ravel()], [p.ravel()], [diag.ravel()]
    for w, di, dj in ((w_xm, -1, 0), (w_xp, 1, 0), (w_zm, 0, -1), (w_zp, 0, 1)):
        ok = (ii + di >= 0) & (ii + di < nx) & (jj + dj >= 0) & (jj + dj < nz)
        rows.append(p[ok])
        cols.append(((jj + dj) * nx + (ii + di))[ok])
        vals.append(w[ok])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nx * nz, nx * nz))
    return A.tocsr()


class BandedLU:
    """LU factorisation with partial pivoting of A in LAPACK band storage.

    The unknowns are reordered so that the shorter grid axis runs fastest,
    giving half-bandwidth min(nx, nz); ``zgbtrf`` factors once and ``zgbtrs``
    solves with A (trans 'N') or with A^H (trans 'C') for any number of
    right-hand sides.  Every source shares the same A, so one factorisation
    serves all K forward and adjoint problems (the block-diagonal structure of
    the stacked system in Section 2).
    """

    def __init__(self, A, nx, nz):
        self.nx, self.nz = nx, nz
        n = nx * nz
        jj, ii = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
        natural = (jj * nx + ii).ravel()
        if nz <= nx:
            banded = (ii * nz + jj).ravel()     # z fastest
            bw = nz
        else:
            banded = natural
            bw = nx
        # perm[q] = natural index of the unknown at banded position q
        perm = np.empty(n, dtype=np.int64)
        perm[banded] = natural
        self.perm = perm
        Ap = A[perm][:, perm].tocoo()
        kl = ku = bw
        ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128)
        ab[kl + ku + Ap.row - Ap.col, Ap.col] = Ap.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv, self.kl, self.ku = lu, piv, kl, ku

    def solve(self, b, adjoint=False):
        """x with A x = b (or A^H x = b); b is [..., nz, nx] or a flat vector."""
        b = np.asarray(b, dtype=np.complex128)
        shape = b.shape
        n = self.nx * self.nz
        B = b.reshape(-1, n).T[self.perm]                  # banded order, one column per RHS
        X, info = lapack.zgbtrs(self.lu, self.kl, self.ku, B, self.piv,
                                trans=2 if adjoint else 0)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        out = np.empty_like(X)
        out[self.perm] = X
        return out.T.reshape(shape)
