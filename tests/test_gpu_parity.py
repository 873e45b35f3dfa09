"""GPU parity of every C-ABI call against the FP64 oracle (MI355X only).

Tolerances: FP64 paths 1e-10 relative (the stated bar; observed ~1e-14 for
operators); complex64 paths are bounded by what FP32 rounding allows, stated
per test.  Sizes are chosen to span several 64 x 4 tiles with ragged tails.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_cases import (oracle_and_gpu, observed_data, eps_rule, to_dev, to_np, rel, tiny_inputs,  # noqa: E402
                             make_problem_inputs)
from synthetic import complex_normal  # noqa: E402

SHAPES = [  # (nx, nz, npml, K)
    dict(nx=21, nz=15, npml=4, K=3),
    dict(nx=133, nz=37, npml=6, K=5),     # ragged against the 64 x 4 tiles
    dict(nx=67, nz=70, npml=5, K=2),      # nz > nx
]


def _case(seed=0, **kw):
    print(f"[case] seed={seed} {kw}", flush=True)
    inp = tiny_inputs(seed=seed, **kw)
    return inp


# 17 sources: the stencil kernel's source groups 0, 1 and a ragged group 2
STENCIL_SHAPES = SHAPES + [dict(nx=133, nz=37, npml=6, K=17)]


@pytest.mark.parametrize("shape", STENCIL_SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_stencil_matches_assembled_matrix(shape, adjoint):
    inp = _case(**shape)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    x = complex_normal(gpu.field_shape, seed=3)
    y = to_np(gpu.stencil_apply(to_dev(x), adjoint=adjoint))
    M = orc.A.conj().T if adjoint else orc.A
    ref = np.stack([M @ x[k].ravel() for k in range(gpu.K)]).reshape(x.shape)
    assert rel(y, ref) <= 1e-13
    y32 = to_np(gpu.stencil_apply(to_dev(x, torch.complex64), adjoint=adjoint))
    assert rel(y32, ref) <= 2e-6


@pytest.mark.parametrize("adjoint", [False, True])
def test_stencil_full_size_matches_assembled_matrix(adjoint):
    """801 x 281 with 80 sources (ten source groups, XCD-contiguous chunks), c128 and c64,
    every output against the oracle's assembled A."""
    from oracle.helmholtz import assemble_A
    from paper_2204_06489_amd.solver import KKTProblem
    inp = make_problem_inputs("c2", 0)
    print(f"[case] stencil 801x281 K=80 adjoint={adjoint}", flush=True)
    gpu = KKTProblem.from_inputs(inp, eps=1.0)
    A = assemble_A(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"], inp["gamma0"],
                   inp["pml_r0"], inp["pml_cref"])
    M = (A.conj().T if adjoint else A).tocsr()
    x = complex_normal(gpu.field_shape, seed=31)
    ref = np.stack([M @ x[k].ravel() for k in range(gpu.K)]).reshape(x.shape)
    y = to_np(gpu.stencil_apply(to_dev(x), adjoint=adjoint))
    assert rel(y, ref) <= 1e-13
    for k in (0, 7, 8, 40, 79):          # per source: no group lost or shifted
        assert rel(y[k], ref[k]) <= 1e-13
    y32 = to_np(gpu.stencil_apply(to_dev(x, torch.complex64), adjoint=adjoint))
    assert rel(y32, ref) <= 2e-6
    for k in (0, 7, 8, 40, 79):
        assert rel(y32[k], ref[k]) <= 2e-6
    gpu.close()


def test_block_solve_largest_batched_grid_matches_banded_lu():
    """The 1001 x 351 grid of the five-frequency batch (10 Hz, 100 sources, 351-row
    columns on the vector units) in c128 and c64, sampled sources against the banded LU."""
    from oracle.kkt import Problem
    from paper_2204_06489_amd.solver import KKTProblem
    inp = make_problem_inputs("c4", 4)
    print(f"[case] block solve {inp['nx']}x{inp['nz']} K={inp['K']} {inp['freq']} Hz", flush=True)
    gpu = KKTProblem.from_inputs(inp, eps=1.0)
    b = complex_normal(gpu.field_shape, seed=41)
    x, st = gpu.helmholtz_solve(to_dev(b), prec="c128", rtol=1e-30)
    x = to_np(x)
    assert st["rel_res_max"] <= 1e-11
    x32, st32 = gpu.helmholtz_solve(to_dev(b, torch.complex64), prec="c64", rtol=1e-30)
    x32 = to_np(x32)
    assert st32["rel_res_max"] <= 1e-3
    gpu.close()
    print("[case] oracle banded LU of 1001x351 ...", flush=True)
    orc = Problem.from_inputs(inp, eps=1.0)
    pick = [0, 1, 37, 63, 99]
    ref = orc.lu.solve(b[pick])
    for i, k in enumerate(pick):
        e64, e32 = rel(x[k], ref[i]), rel(x32[k], ref[i])
        print(f"source {k}: c128 error {e64:.2e}, c64 error {e32:.2e} (c64 residual {st32['rel_res_max']:.1e})")
        assert e64 <= 1e-10
        assert e32 <= 1e-2      # FP32 factors: the residual bound above times the condition number


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_block_solve_matches_banded_lu(shape, adjoint):
    inp = _case(**shape)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    b = complex_normal(gpu.field_shape, seed=5)
    ref = orc.lu.solve(b, adjoint=adjoint)
    x, st = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="c128", rtol=1e-30)
    assert rel(to_np(x), ref) <= 1e-10
    assert st["rel_res_max"] <= 1e-12
    # complex64 factors and buffers: one sweep, FP32 rounding
    x32, st32 = gpu.helmholtz_solve(to_dev(b, torch.complex64), adjoint=adjoint, prec="c64", rtol=1e-30)
    assert st32["rel_res_max"] <= 1e-4
    # complex64 sweeps inside FP64 refinement
    xm, stm = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="mixed", rtol=1e-11, maxit=10)
    assert stm["converged"] and stm["rel_res_max"] <= 1e-11
    assert rel(to_np(xm), ref) <= 1e-9


def test_block_solve_in_place_and_sources():
    inp = _case(**SHAPES[1])
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    f = gpu.sources()
    assert rel(to_np(f), orc.sources()) == 0.0
    u_ref = orc.forward()
    x, _ = gpu.helmholtz_solve(f, out=f)         # rhs and x alias
    assert rel(to_np(x), u_ref) <= 1e-10


def _background(orc, gpu):
    u_n = orc.forward()
    gpu.set_background(to_dev(u_n))
    return u_n


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("weights", ["ones", "random"])
def test_kkt_apply_matches_assembled_kkt_matrix(shape, weights):
    inp = _case(weights=weights, nrec=7, **shape)
    orc, gpu = oracle_and_gpu(inp, eps=3.7e9)
    u_n = _background(orc, gpu)
    xi = complex_normal(orc.nxi, seed=7)
    y = to_np(gpu.kkt_apply(to_dev(xi)))
    ref = orc.kkt_apply(u_n, xi)
    for a, b in zip(orc.unpack(y), orc.unpack(ref)):
        assert rel(a, b) <= 1e-13
    # Hermitian (Section 4): <M x, v> = <x, M v>
    v = complex_normal(orc.nxi, seed=8)
    Mv = to_np(gpu.kkt_apply(to_dev(v)))
    lhs, rhs = np.vdot(y, v), np.vdot(xi, Mv)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_kkt_apply_single_source_group():
    """One source: the matvec kernel forms y_s itself instead of summing group parts."""
    inp = _case(weights="random", nrec=7, nx=133, nz=37, npml=6, K=1)
    orc, gpu = oracle_and_gpu(inp, eps=3.7e9)
    u_n = _background(orc, gpu)
    xi = complex_normal(orc.nxi, seed=11)
    y = to_np(gpu.kkt_apply(to_dev(xi)))
    ref = orc.kkt_apply(u_n, xi)
    for a, b in zip(orc.unpack(y), orc.unpack(ref)):
        assert rel(a, b) <= 1e-13


@pytest.mark.parametrize("cfg,fi", [("c1", 1), ("c2", 0)])
def test_kkt_apply_full_size_matches_oracle(cfg, fi):
    """The workloads bench.py times (401x141 x 40 sources; 801x281 x 80 sources), in the
    launch configuration it times: every output against the oracle's sparse KKT matrix."""
    from oracle.kkt import Problem
    from paper_2204_06489_amd.solver import KKTProblem
    inp = make_problem_inputs(cfg, fi)
    print(f"[case] {cfg} {inp['nx']}x{inp['nz']} K={inp['K']}", flush=True)
    eps = inp["eps"] or 1.0
    orc = Problem.from_inputs(inp, eps=eps, factor=False)
    gpu = KKTProblem.from_inputs(inp, eps=eps)
    u_n = complex_normal((orc.K, orc.nz, orc.nx), seed=21)
    gpu.set_background(to_dev(u_n))
    xi = complex_normal(orc.nxi, seed=22)
    y = to_np(gpu.kkt_apply(to_dev(xi)))
    gpu.close()
    ref = orc.kkt_apply(u_n, xi)
    for a, b in zip(orc.unpack(y), orc.unpack(ref)):
        assert rel(a, b) <= 1e-13


def test_exact_preconditioner_full_size_matches_oracle():
    """The preconditioner at the timed 401x141, 40-source workload (FP64 block solves and
    the stage-2 kernel in the launch configuration bench.py times) against the oracle."""
    from oracle.kkt import Problem
    from paper_2204_06489_amd.solver import KKTProblem
    inp = make_problem_inputs("c1", 1)
    print(f"[case] c1 {inp['nx']}x{inp['nz']} K={inp['K']}", flush=True)
    eps = inp["eps"] or 1.0
    orc = Problem.from_inputs(inp, eps=eps)
    gpu = KKTProblem.from_inputs(inp, eps=eps)
    u_n = complex_normal((orc.K, orc.nz, orc.nx), seed=21)
    gpu.set_background(to_dev(u_n))
    y = complex_normal(orc.nxi, seed=23)
    z = to_np(gpu.precond_apply(to_dev(y), pc="exact"))
    gpu.close()
    ref = orc.precond_apply(u_n, y)
    for a, b in zip(orc.unpack(z), orc.unpack(ref)):
        assert rel(a, b) <= 1e-10


@pytest.mark.parametrize("shape", SHAPES)
def test_exact_preconditioner_matches_oracle_and_inverts(shape):
    inp = _case(nrec=5, **shape)
    orc, gpu = oracle_and_gpu(inp, eps=2.1e9)
    u_n = _background(orc, gpu)
    y = complex_normal(orc.nxi, seed=9)
    z = to_np(gpu.precond_apply(to_dev(y), pc="exact"))
    ref = orc.precond_apply(u_n, y)
    for a, b in zip(orc.unpack(z), orc.unpack(ref)):
        assert rel(a, b) <= 1e-10
    Pm = orc.assemble_M(u_n, W_zero=True)
    assert rel(Pm @ z, y) <= 1e-10


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_inexact_preconditioner_meets_block_bounds(shape):
    """P~ is not unique: check the stage residuals (each block solve with A~ to ~FP32
    accuracy) and that the middle stage is the exact formula given z_lam."""
    inp = _case(nrec=5, **shape)
    orc, gpu = oracle_and_gpu(inp, eps=2.1e9)
    u_n = _background(orc, gpu)
    y = complex_normal(orc.nxi, seed=10)
    z = to_np(gpu.precond_apply(to_dev(y), pc="inexact"))
    yu, ys, yl = orc.unpack(y)
    zu, zs, zl = orc.unpack(z)
    AH = orc.A.conj().T
    for k in range(orc.K):
        assert rel(AH @ zl[k].ravel(), yu[k].ravel()) <= 1e-3
    Pz = np.sum(np.conj(u_n) * zl, axis=0).ravel()[orc.core_idx]
    zs_ref = (ys + orc.omega ** 2 * Pz) / orc.eps
    assert rel(zs, zs_ref) <= 1e-12
    ext = np.zeros(orc.Nu, complex)
    ext[orc.core_idx] = zs
    rhs = yl + orc.omega ** 2 * u_n * ext.reshape(orc.nz, orc.nx)[None]
    for k in range(orc.K):
        assert rel(orc.A @ zu[k].ravel(), rhs[k].ravel()) <= 1e-3


def _newton_setup(K=3, nrec=None, weights="ones", reg=True, **shape):
    inp = _case(K=K, nrec=nrec, weights=weights, **shape)
    d = observed_data(inp)
    orc, gpu = oracle_and_gpu(inp, eps=1.0, reg_on_update=reg)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc.eps = eps
    from paper_2204_06489_amd.solver import KKTProblem
    gpu = KKTProblem.from_inputs(inp, eps=eps, reg_on_update=reg)
    return inp, d, orc, gpu, u_n


@pytest.mark.parametrize("pc", ["exact", "inexact"])
def test_newton_step_matches_exact_kkt_solution(pc):
    """b_s = 0 (the -L s_n := 0 form): the unscaled KKT residual tracks the error, and the FP64
    attainable relative residual is ~1e-12, so tol 1e-11 must give the exact step to 1e-10."""
    inp, d, orc, gpu, u_n = _newton_setup(reg=True, weights="random", nx=41, nz=19, npml=4)
    r = orc.residual(d, u_n)
    xi_ref = orc.kkt_solve_schur(u_n, r)
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-11, restart=40, maxit=200, pc=pc, update_in_place=False)
    assert st["converged"], st
    xi = to_np(xi)
    du, ds, lam = orc.unpack(xi)
    du_r, ds_r, lam_r = orc.unpack(xi_ref)
    errs = (rel(ds, ds_r), rel(du, du_r), rel(lam, lam_r))
    print("errors ds, du, lambda:", errs, "iters", st["outer_iters"])
    assert max(errs) <= 1e-10
    b = orc.rhs(r)
    # backward error recomputed by the oracle (its own FP64 evaluation adds ~1e-12 of rounding)
    bw = rel(orc.kkt_apply(u_n, xi), b)
    print("oracle backward error", bw, "gpu", st["rel_res"])
    assert bw <= 1e-10
    assert max(orc.kkt_rows(u_n, xi, b)) <= 1e-11
    g_ref = orc.update(ds_r)
    assert rel(to_np(g1), g_ref) <= 1e-11
    assert abs(st["misfit_before"] - np.linalg.norm(r) / np.linalg.norm(d)) <= 1e-12
    # the step left gamma_n in place: u_n is the background
    assert rel(to_np(gpu.get_background()), u_n) <= 1e-10


@pytest.mark.parametrize("eta", [1.0, 0.7071067811865476, 0.0])
def test_newton_step_for_every_reorthogonalisation_rule(eta):
    """CGS2 (eta 1), the DGKS test (1/sqrt 2), the default 0.1 and a single classical pass
    (eta 0) all reach the exact step: the basis loses no accuracy that the step sees."""
    inp, d, orc, gpu, u_n = _newton_setup(reg=True, weights="random", nx=41, nz=19, npml=4)
    xi_ref = orc.kkt_solve_schur(u_n, orc.residual(d, u_n))
    xi, _, st = gpu.newton_step(to_dev(d), rtol=1e-11, restart=40, maxit=200, pc="exact", update_in_place=False,
                                reorth_eta=eta)
    assert st["converged"], st
    print(f"eta {eta}: {st['outer_iters']} iterations, {st['reorth_passes']} second passes")
    if eta == 1.0:
        assert st["reorth_passes"] == st["outer_iters"]
    if eta == 0.0:
        assert st["reorth_passes"] == 0
    assert rel(orc.unpack(to_np(xi))[1], orc.unpack(xi_ref)[1]) <= 1e-10


def test_newton_step_rejects_bad_reorthogonalisation_threshold():
    from paper_2204_06489_amd._lib import KFError
    inp, d, orc, gpu, u_n = _newton_setup(reg=True, nx=21, nz=15, npml=4)
    for eta in (-0.1, 1.5, float("nan")):
        with pytest.raises(KFError):
            gpu.newton_step(to_dev(d), rtol=1e-6, reorth_eta=eta)


@pytest.mark.parametrize("pc", ["exact", "inexact"])
def test_newton_step_with_regularisation_row(pc):
    """b_s = -eps s_n (eq. KKT as printed).  ||b|| is then dominated by the control row, so the
    relative residual bounds the data rows only weakly: check the backward error, the two
    exactly resolved first-order rows, and a forward error consistent with it."""
    inp, d, orc, gpu, u_n = _newton_setup(reg=False, weights="random", nx=41, nz=19, npml=4)
    r = orc.residual(d, u_n)
    xi_ref = orc.kkt_solve_schur(u_n, r)
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-12, restart=40, maxit=200, pc=pc, update_in_place=False)
    assert st["converged"], st
    xi = to_np(xi)
    b = orc.rhs(r)
    bw = rel(orc.kkt_apply(u_n, xi), b)
    print("oracle backward error", bw, "gpu", st["rel_res"])
    assert bw <= 1e-11
    rows = orc.kkt_rows(u_n, xi, b)
    assert rows[1] <= 1e-13 and rows[2] <= 1e-10
    assert rel(orc.unpack(xi)[1], orc.unpack(xi_ref)[1]) <= 1e-6


def test_exact_preconditioner_fgmres_terminates_in_rank_F_plus_one():
    inp, d, orc, gpu, u_n = _newton_setup(K=1, nrec=3, nx=21, nz=15, npml=4)
    xi, _, st = gpu.newton_step(to_dev(d), rtol=1e-11, restart=30, maxit=10, pc="exact", update_in_place=False)
    assert st["converged"] and st["outer_iters"] <= 4, st


def test_w_zero_closed_form():
    inp = _case(nx=33, nz=17, npml=4, K=2)
    inp["w"] = np.zeros_like(inp["w"])
    d = observed_data(inp)
    orc, gpu = oracle_and_gpu(inp, eps=0.37, reg_on_update=False)
    u_n = orc.forward()
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-10, restart=10, maxit=20, pc="exact", update_in_place=False)
    du, ds, lam = orc.unpack(to_np(xi))
    assert np.abs(lam).max() <= 1e-12 * max(np.abs(du).max(), 1e-300)
    assert rel(ds, -orc.control()) <= 1e-12
    assert st["outer_iters"] <= 2


def test_reduced_gradient_matches_oracle():
    inp = _case(nx=45, nz=21, npml=5, K=3, weights="random")
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    u = orc.forward()
    from oracle.kkt import adjoint_gradient_full
    c = complex_normal(u.shape, seed=12)
    ref = adjoint_gradient_full(orc.lu, orc.nx, orc.nz, orc.h, orc.npml, orc.omega, u, c, orc.r0, orc.cref)
    g = to_np(gpu.adjoint_gradient(to_dev(u), to_dev(c), prec="c128"))
    assert rel(g, ref) <= 1e-10
    g32 = to_np(gpu.adjoint_gradient(to_dev(u, torch.complex64), to_dev(c, torch.complex64), prec="c64"))
    assert rel(g32, ref) <= 1e-3


def test_c0_newton_step_parity():
    """The c0 workload (101x51, 8 sources, 5 Hz): GPU step vs the oracle's Schur solution."""
    inp = make_problem_inputs("c0")
    print("[case] c0", flush=True)
    d = observed_data(inp)
    orc, gpu = oracle_and_gpu(inp, reg_on_update=True)
    u_n = orc.forward()
    r = orc.residual(d, u_n)
    xi_ref = orc.kkt_solve_schur(u_n, r)
    xi, g1, st = gpu.newton_step(to_dev(d), rtol=1e-11, restart=30, maxit=300, pc="exact", update_in_place=False)
    assert st["converged"], st
    du, ds, lam = orc.unpack(to_np(xi))
    print("c0 ds error", rel(ds, orc.unpack(xi_ref)[1]), "iters", st["outer_iters"])
    assert rel(ds, orc.unpack(xi_ref)[1]) <= 1e-10
    assert rel(to_np(g1), orc.update(orc.unpack(xi_ref)[1])) <= 1e-11
