"""Pins of the oracle's KKT step, preconditioner, gradient and update (CPU only).

The chain of pins: finite differences of the forward map pin the Jacobian
J = Q A^-1 P; numpy's least-squares solver on the GN subproblem pins the normal
equations (H, g); the Schur route pins the dense KKT solve and hence the
assembled KKT matrix; the W = 0 closed form, the preconditioner identities and
the finite-difference gradient pin the remaining pieces.
"""

import numpy as np
import pytest

from oracle.kkt import Problem, gmres_right, adjoint_gradient_full
from tests.oracle_cases import tiny_inputs


def _eps_from_hessian(prob, u_n, rel=1e-2):
    J = prob.jacobians(u_n)
    GN = sum((prob.w[k][:, None] * J[k]).conj().T @ (prob.w[k][:, None] * J[k]) for k in range(prob.K))
    return rel * np.linalg.eigvalsh(GN).max()


def _setup(weights="ones", reg_on_update=False, **kw):
    inp = tiny_inputs(weights=weights, **kw)
    p_true = Problem.from_inputs(inp, gamma=inp["gamma_true"], eps=1.0)
    d = p_true.sample(p_true.forward())
    p = Problem.from_inputs(inp, eps=1.0, reg_on_update=reg_on_update)
    u_n = p.forward()
    p.eps = _eps_from_hessian(p, u_n)
    r = p.residual(d, u_n)
    return p, u_n, r, d


def test_jacobian_matches_forward_map_finite_differences():
    """J dgamma = Q (u(gamma + t dgamma) - u(gamma - t dgamma)) / 2t (eqs. G, S, P, jacobian)."""
    p, u_n, _, _ = _setup()
    J = p.jacobians(u_n)
    rng = np.random.default_rng(11)
    for _ in range(3):
        dg = rng.standard_normal(p.Ng) * np.abs(p.control()).max()
        t = 1e-6
        us = []
        for sgn in (+1, -1):
            g = p.gamma.copy().ravel()
            g[p.core_idx] += sgn * t * dg
            q = Problem(p.nx, p.nz, p.h, p.npml, p.omega, g.reshape(p.nz, p.nx), p.src_ix, p.src_iz,
                        p.rec_ix, p.rec_iz, p.w, p.eps, pml_r0=p.r0, pml_cref=p.cref)
            us.append(q.sample(q.forward()))
        fd = (us[0] - us[1]) / (2 * t)
        lin = np.einsum("krc,c->kr", J, dg)
        assert np.linalg.norm(fd - lin) <= 1e-6 * np.linalg.norm(lin)


@pytest.mark.parametrize("weights", ["ones", "random"])
def test_normal_equations_solve_the_gn_least_squares_problem(weights):
    """ds from (H, g) is the minimiser of 1/2||W(r - J ds)||^2 + eps/2 ||s_n + ds||^2 (eq. tikhonov_discrete),
    computed here by numpy's QR-based least squares on the stacked residual."""
    p, u_n, r, _ = _setup(weights=weights)
    J = p.jacobians(u_n)
    rows = [p.w[k][:, None] * J[k] for k in range(p.K)] + [np.sqrt(p.eps) * np.eye(p.Ng)]
    rhs = [p.w[k] * r[k] for k in range(p.K)] + [-np.sqrt(p.eps) * p.control()]
    ds_ls, *_ = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)
    H, g = p.normal_system(u_n, r)
    ds = np.linalg.solve(H, g)
    assert np.linalg.norm(ds - ds_ls) <= 1e-9 * np.linalg.norm(ds_ls)


@pytest.mark.parametrize("weights,reg", [("ones", False), ("random", False), ("ones", True)])
def test_dense_kkt_equals_schur_route(weights, reg):
    """The KKT solution equals the normal-equation solution (eqs. tmp1, tmp2, normal_system_discrete3)."""
    p, u_n, r, _ = _setup(weights=weights, reg_on_update=reg)
    b = p.rhs(r)
    xi_d = p.kkt_solve_dense(u_n, b)
    xi_s = p.kkt_solve_schur(u_n, r)
    assert np.linalg.norm(xi_d - xi_s) <= 1e-10 * np.linalg.norm(xi_s)
    rows = p.kkt_rows(u_n, xi_s, b)
    assert max(rows) <= 1e-11


def test_kkt_matrix_is_hermitian_and_w_zero_closed_form():
    """M is Hermitian (Section 4); with W = 0 the solution is lambda = 0, ds = -s_n, du = A^-1 P ds."""
    inp = tiny_inputs()
    inp["w"] = np.zeros_like(inp["w"])
    p = Problem.from_inputs(inp, eps=0.37)
    u_n = p.forward()
    M = p.assemble_M(u_n)
    assert abs(M - M.conj().T).max() == 0.0
    b = p.rhs(np.zeros((p.K, p.nrec)))
    xi = p.kkt_solve_dense(u_n, b)
    du, ds, lam = p.unpack(xi)
    assert np.abs(lam).max() <= 1e-12 * np.abs(du).max()
    assert np.linalg.norm(ds + p.control()) <= 1e-12 * np.linalg.norm(p.control())
    ext = np.zeros(p.Nu, complex)
    ext[p.core_idx] = ds
    du_ref = p.lu.solve(p.omega ** 2 * u_n * ext.reshape(p.nz, p.nx)[None])
    assert np.linalg.norm(du - du_ref) <= 1e-10 * np.linalg.norm(du_ref)


def test_preconditioner_inverts_kkt_matrix_without_F():
    """P equals M with F = 0 (eq. precond vs eq. KKT), so P (P^-1 y) = y."""
    p, u_n, _, _ = _setup()
    Pm = p.assemble_M(u_n, W_zero=True)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(p.nxi) + 1j * rng.standard_normal(p.nxi)
    z = p.precond_apply(u_n, y)
    assert np.linalg.norm(Pm @ z - y) <= 1e-10 * np.linalg.norm(y)


def test_exact_preconditioner_gmres_terminates_in_rank_F_plus_one():
    """P^-1 M - I = P^-1 diag(F, 0, 0) has rank <= #receivers, so GMRES with the exact
    preconditioner converges in at most rank(F) + 1 iterations."""
    p, u_n, r, _ = _setup(K=1, nrec=3)
    b = p.rhs(r)
    xi, hist, _ = gmres_right(lambda v: p.kkt_apply(u_n, v), lambda v: p.precond_apply(u_n, v),
                              b, tol=1e-11, restart=30, maxit=10)
    assert len(hist) - 1 <= 4, hist
    xi_s = p.kkt_solve_schur(u_n, r)
    assert np.linalg.norm(xi - xi_s) <= 1e-9 * np.linalg.norm(xi_s)


def test_gmres_iterates_reduce_e_cg_to_zero():
    """E_cg = ||H ds_n - g|| / ||g|| from the GMRES iterates (Section 6) goes to 0 at the solution.

    Uses b_s = 0 (the -L s_n := 0 variant of the multi-frequency experiment), for which the
    KKT residual and E_cg decrease together."""
    p, u_n, r, _ = _setup(reg_on_update=True)
    b = p.rhs(r)
    Hg = p.normal_system(u_n, r)
    xi, hist, its = gmres_right(lambda v: p.kkt_apply(u_n, v), lambda v: p.precond_apply(u_n, v),
                                b, tol=1e-12, restart=40, maxit=80, keep_iterates=True)
    e = [p.e_cg(u_n, r, p.unpack(x)[1], Hg) for x in its]
    assert e[-1] <= 1e-10 and e[0] > 1e-3
    assert hist[-1] <= 1e-12


def test_reduced_gradient_matches_misfit_finite_differences():
    """grad Phi (Section 3 gradient without -L s_n) vs central differences, 20 seeded directions."""
    p, u_n, r, d = _setup(weights="random")
    grad = p.reduced_gradient(u_n, r)
    rng = np.random.default_rng(2)
    s = p.control().real
    for _ in range(20):
        dg = rng.standard_normal(p.Ng)
        t = 1e-6 * np.abs(s).max() / np.abs(dg).max()
        phis = []
        for sgn in (+1, -1):
            g = p.gamma.copy().ravel()
            g[p.core_idx] += sgn * t * dg
            q = Problem(p.nx, p.nz, p.h, p.npml, p.omega, g.reshape(p.nz, p.nx), p.src_ix, p.src_iz,
                        p.rec_ix, p.rec_iz, p.w, p.eps, pml_r0=p.r0, pml_cref=p.cref)
            phis.append(q.misfit(d, q.forward()))
        fd = (phis[0] - phis[1]) / (2 * t)
        # relative to the Cauchy-Schwarz scale |grad| |dg|: a direction nearly
        # orthogonal to the gradient has a tiny derivative that no difference resolves
        assert abs(fd - grad @ dg) <= 1e-6 * np.linalg.norm(grad) * np.linalg.norm(dg)


def test_misfit_taylor_remainder_is_second_order():
    p, u_n, r, d = _setup()
    grad = p.reduced_gradient(u_n, r)
    rng = np.random.default_rng(4)
    dg = rng.standard_normal(p.Ng) * 1e-3 * np.abs(p.control()).max()
    phi0 = p.misfit(d, u_n)
    rem = []
    for t in (1.0, 0.5, 0.25):
        g = p.gamma.copy().ravel()
        g[p.core_idx] += t * dg
        q = Problem(p.nx, p.nz, p.h, p.npml, p.omega, g.reshape(p.nz, p.nx), p.src_ix, p.src_iz,
                    p.rec_ix, p.rec_iz, p.w, p.eps, pml_r0=p.r0, pml_cref=p.cref)
        rem.append(abs(q.misfit(d, q.forward()) - phi0 - t * grad @ dg))
    slopes = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all((slopes > 1.8) & (slopes < 2.2)), slopes


def test_full_grid_adjoint_gradient_matches_finite_differences():
    """d l / d gamma everywhere (PML included) for l = Re<c, u(gamma)>: a plain linear functional."""
    inp = tiny_inputs(K=2)
    p = Problem.from_inputs(inp, eps=1.0)
    u = p.forward()
    rng = np.random.default_rng(9)
    c = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    # l(u) = Re sum conj(c) u  =>  grad_u (dl/dRe u + i dl/dIm u) = c
    grad = adjoint_gradient_full(p.lu, p.nx, p.nz, p.h, p.npml, p.omega, u, c, p.r0, p.cref)
    for _ in range(5):
        dg = rng.standard_normal((p.nz, p.nx)) * np.abs(p.gamma).max()
        t = 1e-6
        ls = []
        for sgn in (+1, -1):
            q = Problem(p.nx, p.nz, p.h, p.npml, p.omega, p.gamma + sgn * t * dg, p.src_ix, p.src_iz,
                        p.rec_ix, p.rec_iz, p.w, p.eps, pml_r0=p.r0, pml_cref=p.cref)
            ls.append(np.real(np.vdot(c, q.forward())))
        fd = (ls[0] - ls[1]) / (2 * t)
        assert abs(fd - np.sum(grad * dg)) <= 1e-6 * np.linalg.norm(grad) * np.linalg.norm(dg)


def test_update_changes_core_only():
    p, u_n, r, _ = _setup()
    xi = p.kkt_solve_schur(u_n, r)
    g1 = p.update(p.unpack(xi)[1])
    assert np.all(g1[~p.core] == p.gamma[~p.core])
    assert np.allclose(g1[p.core], p.gamma[p.core] + np.real(p.unpack(xi)[1]))


@pytest.mark.parametrize("reg", [False, True])
def test_rsgn_cg_converges_to_the_normal_equation_solution(reg):
    """CG on H ds = g (Section 3, Table 1 "CG") reaches the Cholesky solution of the
    normal equations, which numpy's least squares pins; E_cg falls to the tolerance."""
    p, u_n, r, _ = _setup(weights="random", reg_on_update=reg)
    H, g = p.normal_system(u_n, r)
    assert np.linalg.norm(p.gn_gradient(u_n, r) - g) <= 1e-12 * np.linalg.norm(g)
    v = np.random.default_rng(4).standard_normal(p.Ng) + 0j
    assert np.linalg.norm(p.hessian_apply(u_n, v) - H @ v) <= 1e-12 * np.linalg.norm(H @ v)
    ds, hist = p.rsgn_cg(u_n, r, tol=1e-12, maxit=400)
    ref = np.linalg.solve(H, g)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(ds - ref) <= 1e-10 * np.linalg.norm(ref)


def test_real_constrained_step_is_the_real_least_squares_minimiser():
    """The real-constrained GN step minimises 1/2 ||W (r - J ds)||^2 + eps/2 ||ds||^2 over
    real ds (b_s = 0): numpy's least squares on the stacked real and imaginary parts."""
    p, u_n, r, _ = _setup(weights="random", reg_on_update=True)
    J = p.jacobians(u_n)
    WJ = np.vstack([p.w[k][:, None] * J[k] for k in range(p.K)])
    Wr = np.concatenate([p.w[k] * r[k] for k in range(p.K)])
    A_ls = np.vstack([WJ.real, WJ.imag, np.sqrt(p.eps) * np.eye(p.Ng)])
    b_ls = np.concatenate([Wr.real, Wr.imag, np.zeros(p.Ng)])
    ref, *_ = np.linalg.lstsq(A_ls, b_ls, rcond=None)
    ds, hist = p.rsgn_cg(u_n, r, tol=1e-12, maxit=400, real=True)
    assert np.abs(ds.imag).max() == 0.0
    assert np.linalg.norm(ds.real - ref) <= 1e-9 * np.linalg.norm(ref)
    Hr, gr = p.normal_system_real(u_n, r)
    assert np.linalg.norm(np.linalg.solve(Hr, gr) - ref) <= 1e-9 * np.linalg.norm(ref)


def test_continuation_composes_single_steps():
    """The frequency sweep is the composition of exact single steps, each frequency
    starting from the previous one's model; one step at one frequency is the step itself."""
    from oracle.kkt import continuation
    inp = tiny_inputs(weights="random")
    probs, data = [], []
    for f in (4.0, 6.0):
        q = dict(inp, freq=f, omega=2 * np.pi * f)
        pt = Problem.from_inputs(q, gamma=q["gamma_true"], eps=1.0)
        data.append(pt.sample(pt.forward()))
        probs.append(Problem.from_inputs(q, eps=1e3, reg_on_update=True))
    g1, mis = continuation(probs[:1], data[:1], [1])
    p = probs[0]
    u_n = p.forward()
    xi = p.kkt_solve_schur(u_n, p.residual(data[0], u_n))
    assert np.array_equal(g1, p.update(p.unpack(xi)[1]))
    g2, mis2 = continuation(probs, data, [1, 2])
    q = probs[1].with_gamma(g1)
    for _ in range(2):
        u = q.forward()
        q = q.with_gamma(q.update(q.unpack(q.kkt_solve_schur(u, q.residual(data[1], u)))[1]))
    assert np.array_equal(g2, q.gamma)
    assert len(mis2) == 3


def test_lbfgs_inverse_meets_the_secant_condition_and_reduces_to_L():
    """The L-BFGS H-block: without pairs it is L^-1 = I / eps; with pairs of the true
    Hessian it maps the newest y to its s (the secant condition) and stays Hermitian
    positive definite."""
    p, u_n, r, _ = _setup(weights="random")
    rng = np.random.default_rng(12)
    q = rng.standard_normal(p.Ng) + 1j * rng.standard_normal(p.Ng)
    assert np.array_equal(p.lbfgs_inverse(q, []), q / p.eps)
    H, _ = p.normal_system(u_n, r)
    pairs = []
    for _ in range(3):
        s = rng.standard_normal(p.Ng) + 1j * rng.standard_normal(p.Ng)
        pairs.append((s, H @ s))
    s3, y3 = pairs[-1]
    assert np.linalg.norm(p.lbfgs_inverse(y3, pairs) - s3) <= 1e-10 * np.linalg.norm(s3)
    B = np.stack([p.lbfgs_inverse(e, pairs) for e in np.eye(p.Ng)], axis=1)
    assert np.abs(B - B.conj().T).max() <= 1e-10 * np.abs(B).max()
    assert np.linalg.eigvalsh((B + B.conj().T) / 2).min() > 0
    y = rng.standard_normal(p.nxi) + 1j * rng.standard_normal(p.nxi)
    z0 = p.precond_apply_hblock(u_n, y, [])
    assert np.linalg.norm(z0 - p.precond_apply(u_n, y)) <= 1e-12 * np.linalg.norm(z0)
