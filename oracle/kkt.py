"""Full-space Gauss-Newton KKT step, plain FP64 (oracle; test infrastructure only).

Follows Sections 3-5 of the paper:

* the GN subproblem for the update ds (eq. tikhonov_discrete) with data residual
  r = d - Q S(s_n), real diagonal weights W and L = eps I;
* the Frechet derivative G = A^-1 P with P = omega^2 diag(u_n) (eqs. G, S, P), the
  Jacobian J = Q A^-1 P, the Hessian H = J^* W^T W J + L and gradient
  g = J^* W^T W r - L s_n (Section 3; the W placement is read from the KKT
  right-hand side b_1 = Q^* W^T W r);
* the KKT system M xi = b (eq. KKT) with xi = (du, ds, lambda) stacked over
  sources (eq. partitioned_system_matrix);
* its equivalence with the normal equations (eqs. tmp1, tmp2,
  normal_system_discrete3, with W kept in tmp2);
* the block-triangular preconditioner (eq. precond) and GMRES on the
  preconditioned system (Section 5).

The control s is the squared slowness on the core nodes; E extends a core
vector to the full grid (zero in the PML), so P_k = omega^2 diag(u_k) E.
Packed vectors are [du_0 .. du_{K-1} | ds | lambda_0 .. lambda_{K-1}] with each
field [nz][nx] and ds [nz - 2 npml][nx - 2 npml].
"""

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

from .helmholtz import assemble_A, BandedLU
from .pml import core_mask


class Problem:
    """One (grid, frequency, geometry) instance with its assembled A and LU.

    ``gamma`` is the full-grid squared slowness [nz][nx]; its core part is the
    control s_n.  ``w`` is [K][nrec] (receiver weights of each source).
    """

    def __init__(self, nx, nz, h, npml, omega, gamma, src_ix, src_iz, rec_ix, rec_iz,
                 w=None, eps=1.0, reg_on_update=False, pml_r0=1e-3, pml_cref=4000.0,
                 factor=True):
        self.nx, self.nz, self.h, self.npml, self.omega = nx, nz, float(h), npml, float(omega)
        self.gamma = np.array(gamma, dtype=np.float64)
        self.src_ix = np.asarray(src_ix, dtype=np.int64)
        self.src_iz = np.asarray(src_iz, dtype=np.int64)
        self.rec_ix = np.asarray(rec_ix, dtype=np.int64)
        self.rec_iz = np.asarray(rec_iz, dtype=np.int64)
        self.K = len(self.src_ix)
        self.nrec = len(self.rec_ix)
        self.w = np.ones((self.K, self.nrec)) if w is None else np.asarray(w, dtype=np.float64)
        self.eps = float(eps)
        self.reg_on_update = bool(reg_on_update)
        self.r0, self.cref = pml_r0, pml_cref
        self.Nu = nx * nz
        self.core = core_mask(nx, nz, npml)
        self.core_idx = np.flatnonzero(self.core.ravel())      # natural index of each control node
        self.Ng = self.core_idx.size
        self.A = assemble_A(nx, nz, h, npml, omega, self.gamma, pml_r0, pml_cref)
        self.lu = BandedLU(self.A, nx, nz) if factor else None

    @classmethod
    def from_inputs(cls, inp, gamma=None, eps=None, K=None, **kw):
        g = inp["gamma0"] if gamma is None else gamma
        K = inp["K"] if K is None else K
        return cls(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], g,
                   inp["src_ix"][:K], inp["src_iz"][:K], inp["rec_ix"], inp["rec_iz"],
                   w=inp["w"][:K], eps=inp["eps"] if eps is None else eps,
                   pml_r0=inp["pml_r0"], pml_cref=inp["pml_cref"], **kw)

    def with_gamma(self, gamma, omega=None):
        """The same grid, acquisition, weights and eps with another gamma (and frequency)."""
        return Problem(self.nx, self.nz, self.h, self.npml, self.omega if omega is None else omega, gamma,
                       self.src_ix, self.src_iz, self.rec_ix, self.rec_iz, w=self.w, eps=self.eps,
                       reg_on_update=self.reg_on_update, pml_r0=self.r0, pml_cref=self.cref)

    # --- sizes and packing -------------------------------------------------
    @property
    def nxi(self):
        return 2 * self.K * self.Nu + self.Ng

    def pack(self, du, ds, lam):
        return np.concatenate([np.ravel(du), np.ravel(ds), np.ravel(lam)]).astype(np.complex128)

    def unpack(self, xi):
        n = self.K * self.Nu
        du = xi[:n].reshape(self.K, self.nz, self.nx)
        ds = xi[n:n + self.Ng]
        lam = xi[n + self.Ng:].reshape(self.K, self.nz, self.nx)
        return du, ds, lam

    def control(self):
        """s_n: the core part of gamma as a flat vector."""
        return self.gamma.ravel()[self.core_idx].astype(np.complex128)

    # --- sources, observation, weights (Section 2 observation operator; eq. tikhonov_discrete W)
    def sources(self):
        """f_k = e_{src_k} / h^2: a unit discrete delta at each source node, [K][nz][nx]."""
        f = np.zeros((self.K, self.nz, self.nx), dtype=np.complex128)
        f[np.arange(self.K), self.src_iz, self.src_ix] = 1.0 / self.h ** 2
        return f

    def Q(self):
        """Receiver sampling matrix [nrec x Nu] (Dirac receivers on grid nodes)."""
        cols = self.rec_iz * self.nx + self.rec_ix
        return sp.csr_matrix((np.ones(self.nrec), (np.arange(self.nrec), cols)),
                             shape=(self.nrec, self.Nu))

    def E(self):
        """Extension from core control nodes to the full grid [Nu x Ng]."""
        return sp.csr_matrix((np.ones(self.Ng), (self.core_idx, np.arange(self.Ng))),
                             shape=(self.Nu, self.Ng))

    def sample(self, u):
        """d_k = Q u_k for every source: [K][nrec]."""
        return np.asarray(u).reshape(self.K, -1)[:, self.rec_iz * self.nx + self.rec_ix]

    # --- forward problem and residual (Section 3: u = S(s), r = d - Q S(s_n))
    def forward(self):
        return self.lu.solve(self.sources())

    def residual(self, d, u):
        return np.asarray(d) - self.sample(u)

    def misfit(self, d, u):
        """Phi = 1/2 sum_k ||W_k (d_k - Q u_k)||^2 (the data term of the GN objective)."""
        r = self.residual(d, u)
        return 0.5 * float(np.sum(np.abs(self.w * r) ** 2))

    # --- the KKT matrix and right-hand side (eq. KKT, eq. partitioned_system_matrix)
    def blocks(self, u_n):
        """(F, A_blk, P) for the stacked sources; F_k = Q^T W_k^2 Q, P_k = omega^2 diag(u_k) E."""
        Q = self.Q()
        E = self.E()
        F = sp.block_diag([Q.T @ sp.diags(self.w[k] ** 2) @ Q for k in range(self.K)])
        A_blk = sp.block_diag([self.A] * self.K)
        u_n = np.asarray(u_n).reshape(self.K, -1)
        P = sp.vstack([self.omega ** 2 * sp.diags(u_n[k]) @ E for k in range(self.K)])
        return F.tocsr(), A_blk.tocsr(), P.tocsr()

    def assemble_M(self, u_n, W_zero=False):
        """The KKT matrix M = [[F, 0, A^*], [0, L, -P^*], [A, -P, 0]] as sparse CSR.

        With ``W_zero`` the F block is dropped, which is exactly the
        preconditioner of eq. precond (M with F = 0)."""
        F, A_blk, P = self.blocks(u_n)
        if W_zero:
            F = sp.csr_matrix(F.shape, dtype=np.complex128)
        L = self.eps * sp.identity(self.Ng, dtype=np.complex128, format="csr")
        M = sp.bmat([[F, None, A_blk.conj().T],
                     [None, L, -P.conj().T],
                     [A_blk, -P, None]], format="csr")
        return M

    def rhs(self, r):
        """b = [Q^* W^T W r ; -L s_n ; 0] (eq. KKT); -L s_n is 0 with reg_on_update."""
        Q = self.Q()
        r = np.asarray(r).reshape(self.K, self.nrec)
        bu = np.stack([Q.T @ (self.w[k] ** 2 * r[k]) for k in range(self.K)])
        bs = np.zeros(self.Ng, np.complex128) if self.reg_on_update else -self.eps * self.control()
        return self.pack(bu, bs, np.zeros_like(bu))

    def kkt_apply(self, u_n, xi):
        """y = M xi with the assembled matrix."""
        return self.assemble_M(u_n) @ np.asarray(xi, dtype=np.complex128)

    # --- block-triangular preconditioner (eq. precond) ------------------------
    def precond_apply(self, u_n, y):
        """z = P^-1 y for P = [[0, 0, A^*], [0, L, -P^*], [A, -P, 0]].

        Row 1: A^* z_lam = y_u; row 2: L z_s - P^* z_lam = y_s;
        row 3: A z_u - P z_s = y_lam.  Solved in that order with the banded LU."""
        yu, ys, ylam = self.unpack(np.asarray(y, dtype=np.complex128))
        u_n = np.asarray(u_n).reshape(self.K, self.nz, self.nx)
        w2 = self.omega ** 2
        z_lam = self.lu.solve(yu, adjoint=True)
        Pz = np.sum(np.conj(u_n) * z_lam, axis=0).ravel()[self.core_idx]   # sum_k P_k^* z_lam,k / w^2
        z_s = (ys + w2 * Pz) / self.eps
        ext = np.zeros(self.Nu, np.complex128)
        ext[self.core_idx] = z_s
        rhs_u = ylam + w2 * u_n * ext.reshape(self.nz, self.nx)[None]
        z_u = self.lu.solve(rhs_u)
        return self.pack(z_u, z_s, z_lam)

    def lbfgs_inverse(self, q, pairs):
        """Ht^-1 q for the L-BFGS approximation Ht of the reduced Hessian with L = eps I as
        the initial matrix (Section 5: an approximation of H in place of L in the middle
        stage), by the two-loop recursion over the pairs (s_i, y_i = H s_i), oldest first,
        with the curvature Re(y_i^H s_i) (H is Hermitian)."""
        q = np.array(q, dtype=np.complex128)
        a = []
        for s_i, y_i in reversed(pairs):
            rho = 1.0 / np.real(np.vdot(y_i, s_i))
            a_i = rho * np.vdot(s_i, q)
            a.append((a_i, rho))
            q = q - a_i * y_i
        r = q / self.eps
        for (s_i, y_i), (a_i, rho) in zip(pairs, reversed(a)):
            b = rho * np.vdot(y_i, r)
            r = r + (a_i - b) * s_i
        return r

    def precond_apply_hblock(self, u_n, y, pairs):
        """The block-triangular preconditioner with the L-BFGS H-block in the middle
        stage: z_lam = A^-* y_u, z_s = Ht^-1 (y_s + P^* z_lam), z_u = A^-1 (y_lam + P z_s)."""
        yu, ys, ylam = self.unpack(np.asarray(y, dtype=np.complex128))
        u_n = np.asarray(u_n).reshape(self.K, self.nz, self.nx)
        w2 = self.omega ** 2
        z_lam = self.lu.solve(yu, adjoint=True)
        q = ys + w2 * np.sum(np.conj(u_n) * z_lam, axis=0).ravel()[self.core_idx]
        z_s = self.lbfgs_inverse(q, pairs)
        ext = np.zeros(self.Nu, np.complex128)
        ext[self.core_idx] = z_s
        z_u = self.lu.solve(ylam + w2 * u_n * ext.reshape(self.nz, self.nx)[None])
        return self.pack(z_u, z_s, z_lam)

    # --- exact solutions ---------------------------------------------------------
    def kkt_solve_dense(self, u_n, b):
        """xi = M^-1 b by dense LU of the assembled KKT matrix (tiny grids only)."""
        M = self.assemble_M(u_n).toarray()
        return np.linalg.solve(M, b)

    def jacobians(self, u_n):
        """J_k = Q A^-1 P_k for every source, as a [K][nrec][Ng] array.

        The receivers are shared by all sources, so G = A^-* Q^T (nrec adjoint
        solves) gives every J_k = G^* P_k (eq. jacobian)."""
        Qd = self.Q().T.toarray().T.reshape(self.nrec, self.nz, self.nx).astype(np.complex128)
        G = self.lu.solve(Qd, adjoint=True).reshape(self.nrec, -1)      # rows: (A^-* q_r)^T
        u_n = np.asarray(u_n).reshape(self.K, -1)
        Gc = np.conj(G[:, self.core_idx])                               # (G^*)[r, core]
        return self.omega ** 2 * Gc[None, :, :] * u_n[:, self.core_idx][:, None, :]

    def gn_operator(self, u_n):
        """v -> sum_k J_k^* W_k^2 J_k v without forming J (Hessian of Section 3 without L).

        Uses G = A^-* Q^T (nrec adjoint solves, shared by all sources):
        J_k v = omega^2 conj(G_core) (u_k * v) and J_k^* y = omega^2 conj(u_k) * (G_core^T y)."""
        Qd = self.Q().toarray().reshape(self.nrec, self.nz, self.nx).astype(np.complex128)
        Gc = self.lu.solve(Qd, adjoint=True).reshape(self.nrec, -1)[:, self.core_idx]
        uc = np.asarray(u_n).reshape(self.K, -1)[:, self.core_idx]
        w2 = self.omega ** 2

        def apply(v):
            out = np.zeros(self.Ng, np.complex128)
            for k in range(self.K):
                y = w2 * (np.conj(Gc) @ (uc[k] * v))
                out += w2 * np.conj(uc[k]) * (Gc.T @ (self.w[k] ** 2 * y))
            return out
        return apply

    def normal_system(self, u_n, r):
        """(H, g) with H = sum_k J_k^* W_k^2 J_k + eps I and g = sum_k J_k^* W_k^2 r_k - L s_n."""
        J = self.jacobians(u_n)
        r = np.asarray(r).reshape(self.K, self.nrec)
        H = self.eps * np.eye(self.Ng, dtype=np.complex128)
        g = np.zeros(self.Ng, np.complex128) if self.reg_on_update else -self.eps * self.control()
        for k in range(self.K):
            WJ = self.w[k][:, None] * J[k]
            H += WJ.conj().T @ WJ
            g += J[k].conj().T @ (self.w[k] ** 2 * r[k])
        return H, g

    def kkt_solve_schur(self, u_n, r):
        """Exact xi through the normal equations (eqs. tmp1, tmp2, normal_system_discrete3).

        ds = H^-1 g (Cholesky), du_k = A^-1 P_k ds,
        lambda_k = A^-* Q^T W_k^2 (r_k - Q du_k)."""
        H, g = self.normal_system(u_n, r)
        c, low = sla.cho_factor(H)
        ds = sla.cho_solve((c, low), g)
        u_n = np.asarray(u_n).reshape(self.K, self.nz, self.nx)
        ext = np.zeros(self.Nu, np.complex128)
        ext[self.core_idx] = ds
        du = self.lu.solve(self.omega ** 2 * u_n * ext.reshape(self.nz, self.nx)[None])
        rr = np.asarray(r).reshape(self.K, self.nrec) - self.sample(du)
        Q = self.Q()
        src = np.stack([Q.T @ (self.w[k] ** 2 * rr[k]) for k in range(self.K)])
        lam = self.lu.solve(src.reshape(self.K, self.nz, self.nx), adjoint=True)
        return self.pack(du, ds, lam)

    def kkt_rows(self, u_n, xi, b):
        """Backward errors of the three first-order conditions (Section 4, the KKT
        system) at xi.  Row block t gives ||b_t - (M xi)_t|| / (||(|M| |xi|)_t|| + ||b_t||):
        the blocks differ in scale by many orders of magnitude (the control row
        carries eps ~ |J|^2), so each is measured against its own terms."""
        M = self.assemble_M(u_n)
        xi = np.asarray(xi, dtype=np.complex128)
        res = self.unpack(b - M @ xi)
        mag = self.unpack(abs(M) @ np.abs(xi) + 0j)
        bb = self.unpack(np.asarray(b))
        return tuple(np.linalg.norm(res[t]) / (np.linalg.norm(mag[t]) + np.linalg.norm(bb[t]))
                     for t in range(3))

    def e_cg(self, u_n, r, ds, H_g=None):
        """E_cg = ||H ds - g|| / ||g|| (Section 6, the CG error measure)."""
        H, g = self.normal_system(u_n, r) if H_g is None else H_g
        return np.linalg.norm(H @ ds - g) / np.linalg.norm(g)

    # --- reduced-space Gauss-Newton by CG (Section 3, the RSGN-CG baseline) ------
    def gn_gradient(self, u_n, r):
        """g = sum_k J_k^* W_k^2 r_k - L s_n (Section 3; -L s_n dropped with reg_on_update),
        from one adjoint solve per source: J_k^* y = omega^2 E^T conj(u_k) (A^-* Q^T y)."""
        Q = self.Q()
        r = np.asarray(r).reshape(self.K, self.nrec)
        src = np.stack([Q.T @ (self.w[k] ** 2 * r[k]) for k in range(self.K)])
        lam0 = self.lu.solve(src.reshape(self.K, self.nz, self.nx), adjoint=True)
        u = np.asarray(u_n).reshape(self.K, -1)
        g = self.omega ** 2 * np.sum(np.conj(u) * lam0.reshape(self.K, -1), axis=0)[self.core_idx]
        if not self.reg_on_update:
            g = g - self.eps * self.control()
        return g

    def hessian_apply(self, u_n, v):
        """H v = L v + sum_k J_k^* W_k^2 J_k v with L = eps I, by two solves per source
        (Section 3): du_k = A^-1 P_k v, lambda_k = A^-* Q^T W_k^2 Q du_k,
        H v = eps v + omega^2 E^T sum_k conj(u_k) lambda_k."""
        u = np.asarray(u_n).reshape(self.K, self.nz, self.nx)
        ext = np.zeros(self.Nu, np.complex128)
        ext[self.core_idx] = v
        du = self.lu.solve(self.omega ** 2 * u * ext.reshape(self.nz, self.nx)[None])
        Q = self.Q()
        src = np.stack([Q.T @ (self.w[k] ** 2 * (Q @ du[k].ravel())) for k in range(self.K)])
        lam = self.lu.solve(src.reshape(self.K, self.nz, self.nx), adjoint=True)
        return self.eps * v + self.omega ** 2 * np.sum(np.conj(u) * lam, axis=0).ravel()[self.core_idx]

    def rsgn_cg(self, u_n, r, tol=1e-8, maxit=500, real=False):
        """Conjugate gradients on the normal equations H ds = g (Section 3, the reduced-space
        Gauss-Newton step the paper compares with; Table 1 "CG").  The iteration stops
        when ||H ds - g|| <= tol ||g|| (E_cg of Section 6).

        real=True solves the real-constrained step instead: ds real with
        Re(H) ds = Re(g), the normal equations of the GN problem over real updates
        (for real v, Re(H v) = Re(H) v since L is real).
        Returns (ds, history of ||H ds - g|| / ||g||)."""
        g = self.gn_gradient(u_n, r)
        if real:
            g = g.real.astype(np.complex128)
        apply = (lambda v: self.hessian_apply(u_n, v).real.astype(np.complex128)) if real else \
            (lambda v: self.hessian_apply(u_n, v))
        x = np.zeros_like(g)
        res = g.copy()
        d = res.copy()
        rr = np.real(np.vdot(res, res))
        gn = np.sqrt(rr)
        hist = [1.0]
        for _ in range(maxit):
            if np.sqrt(rr) <= tol * gn:
                break
            Hd = apply(d)
            alpha = rr / np.real(np.vdot(d, Hd))
            x = x + alpha * d
            res = res - alpha * Hd
            rr_new = np.real(np.vdot(res, res))
            d = res + (rr_new / rr) * d
            rr = rr_new
            hist.append(np.sqrt(rr) / gn)
        return x, hist

    def normal_system_real(self, u_n, r):
        """(Re H, Re g): the normal equations of the GN step restricted to real ds."""
        H, g = self.normal_system(u_n, r)
        return H.real, g.real

    # --- reduced gradient and update ------------------------------------------
    def reduced_gradient(self, u_n, r):
        """grad Phi on the core: -omega^2 sum_k Re(conj(u_k) * lambda0_k),
        lambda0_k = A^-* Q^T W_k^2 r_k (the gradient of Section 3 without -L s_n)."""
        Q = self.Q()
        r = np.asarray(r).reshape(self.K, self.nrec)
        src = np.stack([Q.T @ (self.w[k] ** 2 * r[k]) for k in range(self.K)])
        lam0 = self.lu.solve(src.reshape(self.K, self.nz, self.nx), adjoint=True)
        u_n = np.asarray(u_n).reshape(self.K, -1)
        return -self.omega ** 2 * np.sum(np.real(np.conj(u_n) * lam0.reshape(self.K, -1)),
                                         axis=0)[self.core_idx]

    def update(self, ds):
        """gamma_{n+1} = gamma_n + Re(ds) on the core; PML values unchanged (s_{n+1} = s_n + ds)."""
        g = self.gamma.copy().ravel()
        g[self.core_idx] += np.real(ds)
        return g.reshape(self.nz, self.nx)


def continuation(problems, data, steps):
    """Frequency continuation (Section 6, the frequency sweep): the problems (same grid,
    increasing frequency, each with its own eps) are inverted in order, steps[q] exact
    Newton steps each (the Schur route of eqs. tmp1, tmp2, normal_system_discrete3 and
    the update s_{n+1} = s_n + Re(ds)), every problem starting from the model the
    previous one reached.  Returns (final gamma, misfits ||d - Q u_n|| / ||d|| before
    every step)."""
    gamma = problems[0].gamma
    misfits = []
    for prob, d, n in zip(problems, data, steps):
        p = prob.with_gamma(gamma)
        for _ in range(n):
            u_n = p.forward()
            r = p.residual(d, u_n)
            misfits.append(np.linalg.norm(r) / np.linalg.norm(d))
            xi = p.kkt_solve_schur(u_n, r)
            gamma = p.update(p.unpack(xi)[1])
            p = p.with_gamma(gamma)
    return gamma, misfits


def adjoint_gradient_full(A_solver, nx, nz, h, npml, omega, u, grad_u, r0, cref):
    """d loss / d gamma on the full grid for u = A(gamma)^-1 f.

    With grad_u = dl/dRe(u) + i dl/dIm(u) and mu = A^-* grad_u, the chain rule
    through dA/dgamma = -omega^2 X Z (the mass term of the PML Helmholtz
    operator) gives dl/dgamma = omega^2 sum_k Re(conj(mu_k) X Z u_k).  On the
    core X = Z = 1 and this is the reduced gradient of Section 3."""
    from .pml import stretch
    Xn, _ = stretch(nx, h, npml, omega, r0, cref)
    Zn, _ = stretch(nz, h, npml, omega, r0, cref)
    XZ = Zn[:, None] * Xn[None, :]
    mu = A_solver.solve(grad_u, adjoint=True)
    return omega ** 2 * np.sum(np.real(np.conj(mu) * XZ[None] * u), axis=0)


def gmres_right(apply_M, apply_Pinv, b, tol=1e-12, restart=30, maxit=500, keep_iterates=False):
    """Right-preconditioned restarted GMRES for M xi = b (Section 5, FSGN-GMRes).

    Minimises ||b - M xi||_2 (the E_gmres quantity of Section 6) over
    xi = xi0 + Z y with Z the preconditioned Arnoldi basis; modified
    Gram-Schmidt; starts from xi = 0; stops when ||b - M xi|| <= tol ||b||.
    Returns (xi, history of relative residual estimates, iterates or None)."""
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    xi = np.zeros_like(b)
    hist = [1.0]
    iterates = [] if keep_iterates else None
    if nb == 0.0:
        return xi, hist, iterates
    total = 0
    while total < maxit:
        r = b - apply_M(xi) if total else b.copy()
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            break
        V = [r / beta]
        Z = []
        Hm = np.zeros((restart + 1, restart), dtype=np.complex128)
        for j in range(restart):
            Z.append(apply_Pinv(V[j]))
            w = apply_M(Z[j])
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            total += 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(Hm[:j + 2, :j + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - Hm[:j + 2, :j + 1] @ y)
            hist.append(res / nb)
            if keep_iterates:
                iterates.append(xi + sum(y[i] * Z[i] for i in range(j + 1)))
            if res <= tol * nb or Hm[j + 1, j] == 0.0 or total >= maxit:
                break
            V.append(w / Hm[j + 1, j])
        xi = xi + sum(y[i] * Z[i] for i in range(len(y)))
        if hist[-1] <= tol:
            break
    return xi, hist, iterates
