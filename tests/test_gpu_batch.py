"""GPU tests of batches: several problems on uneven grids in persistent launches.

Each problem of a batch must give what it gives alone (same kernels; the batch's
launch shape may change the rounding order, so 1e-12) and what the oracle gives."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd.solver import KKTBatch, KKTProblem  # noqa: E402
from synthetic import complex_normal  # noqa: E402
from tests.gpu_cases import eps_rule, observed_data, oracle_and_gpu, rel, to_dev, to_np  # noqa: E402
from tests.oracle_cases import tiny_inputs  # noqa: E402

SHAPES = [dict(nx=21, nz=15, npml=4, K=3, freq=4.0), dict(nx=41, nz=19, npml=4, K=2, freq=6.0),
          dict(nx=67, nz=37, npml=5, K=4, freq=8.0)]


def _cases(weights="ones"):
    out = []
    for q, sh in enumerate(SHAPES):
        print(f"[case] batch member {q}: {sh}", flush=True)
        inp = tiny_inputs(seed=q, weights=weights, **sh)
        out.append(inp)
    return out


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_batched_solve_matches_single_problem_solves(prec, adjoint):
    inps = _cases()
    pairs = [oracle_and_gpu(inp, eps=1.0) for inp in inps]
    gpus = [g for _, g in pairs]
    dt = torch.complex64 if prec == "c64" else torch.complex128
    rhs = [to_dev(complex_normal(g.field_shape, seed=20 + q), dt) for q, g in enumerate(gpus)]
    singles = [g.helmholtz_solve(r, adjoint=adjoint, prec=prec)[0] for g, r in zip(gpus, rhs)]
    batch = KKTBatch(gpus)
    xs = batch.helmholtz_solve(rhs, adjoint=adjoint, prec=prec)
    for (orc, g), x, s1, r in zip(pairs, xs, singles, rhs):
        assert rel(to_np(x), to_np(s1)) <= (1e-12 if prec == "c128" else 1e-5)
        if prec == "c128":
            assert rel(to_np(x), orc.lu.solve(to_np(r), adjoint=adjoint)) <= 1e-10
    batch.close()


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("pc", ["exact", "inexact"])
def test_batched_newton_step_matches_oracle(use_graph, pc):
    inps = _cases(weights="random")
    gpus, orcs, ds, refs = [], [], [], []
    for inp in inps:
        d = observed_data(inp)
        orc, _ = oracle_and_gpu(inp, eps=1.0)
        u_n = orc.forward()
        orc.eps = eps_rule(orc, u_n)
        gpus.append(KKTProblem.from_inputs(inp, eps=orc.eps))
        orcs.append(orc)
        ds.append(to_dev(d))
        refs.append(orc.kkt_solve_schur(u_n, orc.residual(d, u_n)))
    batch = KKTBatch(gpus)
    xis, gs, sts = batch.newton_step(ds, rtol=1e-11, restart=15, maxit=300, pc=pc, update_in_place=False,
                                     use_graph=use_graph)
    for orc, xi, g1, st, ref in zip(orcs, xis, gs, sts, refs):
        assert st["converged"], st
        err = rel(orc.unpack(to_np(xi))[1], orc.unpack(ref)[1])
        print(f"member ds error {err:.2e}, {st['outer_iters']} iterations, {st['restarts']} cycles")
        assert err <= 1e-10
        assert rel(to_np(g1), orc.update(orc.unpack(ref)[1])) <= 1e-11
    # a second step with graphs replays the captured columns (same factors, same pointers)
    if use_graph:
        xis2, _, sts2 = batch.newton_step(ds, rtol=1e-11, restart=15, maxit=300, pc=pc, update_in_place=False,
                                          use_graph=True)
        for xi, xi2 in zip(xis, xis2):
            assert rel(to_np(xi2), to_np(xi)) <= 1e-13
    batch.close()


def test_problems_work_alone_after_their_batch_is_destroyed():
    """The batch lends its stream to its members; destroying it hands each member its own
    stream back, so a later single-problem call still launches (same result as batched)."""
    inps = _cases(weights="random")[:2]
    gpus, ds = [], []
    for inp in inps:
        ds.append(to_dev(observed_data(inp)))
        orc, _ = oracle_and_gpu(inp, eps=1.0)
        gpus.append(KKTProblem.from_inputs(inp, eps=eps_rule(orc, orc.forward())))
    batch = KKTBatch(gpus)
    xis, _, sts = batch.newton_step(ds, rtol=1e-11, restart=15, maxit=300, pc="exact", update_in_place=False,
                                    use_graph=True)
    assert all(st["converged"] for st in sts)
    xis = [x.clone() for x in xis]
    batch.close()
    torch.cuda.synchronize()
    for g, d, xb in zip(gpus, ds, xis):
        xi, _, st = g.newton_step(d, rtol=1e-11, restart=15, maxit=300, pc="exact", update_in_place=False)
        assert st["converged"]
        assert rel(to_np(xi), to_np(xb)) <= 1e-10


def test_batch_mixing_sweep_kernels_matches_single_problem_solves():
    """Members whose columns take different complex64 sweep kernels (matrix cores with one
    or two row tiles per wavefront, vector units above 288 rows) share one batch."""
    shapes = [dict(nx=21, nz=19, npml=4, K=3, freq=6.0), dict(nx=21, nz=150, npml=4, K=2, freq=6.0),
              dict(nx=21, nz=300, npml=4, K=2, freq=6.0)]
    gpus, rhs = [], []
    for q, sh in enumerate(shapes):
        print(f"[case] mixed-kernel batch member {q}: {sh}", flush=True)
        g = KKTProblem.from_inputs(tiny_inputs(seed=q, **sh), eps=1.0)
        gpus.append(g)
        rhs.append(to_dev(complex_normal(g.field_shape, seed=40 + q), torch.complex64))
    singles = [g.helmholtz_solve(r, prec="c64")[0] for g, r in zip(gpus, rhs)]
    batch = KKTBatch(gpus)
    xs = batch.helmholtz_solve(rhs, prec="c64")
    # the members' own calls below run on their own streams again (ordered with torch's)
    batch.close()
    for g, x, s1, r in zip(gpus, xs, singles, rhs):
        x64, r64 = x.to(torch.complex128), r.to(torch.complex128)
        xref = g.helmholtz_solve(r64, prec="c128")[0]
        res = rel(to_np(g.stencil_apply(x64)), to_np(r64))
        res_ref = rel(to_np(g.stencil_apply(xref)), to_np(r64))
        print(f"member nz={g.nz}: batch vs single {rel(to_np(x), to_np(s1)):.1e}, residual {res:.1e} "
              f"(c128 solve {res_ref:.1e}), vs c128 solve {rel(to_np(x64), to_np(xref)):.1e}, "
              f"|x| {float(x64.abs().max()):.2e}", flush=True)
        assert rel(to_np(x), to_np(s1)) <= 1e-5
        assert rel(to_np(x64), to_np(xref)) <= 1e-3


def test_batch_mixing_fp64_sweep_kernels_matches_single_problem_solves():
    """The same mixed batch in FP64: the members' columns take the FP64 matrix-core sweeps
    with three or six wavefronts, or the vector units above 288 rows, with three chunks
    each (spikes, reduction and interior correction in every member)."""
    shapes = [dict(nx=21, nz=19, npml=4, K=3, freq=6.0), dict(nx=21, nz=150, npml=4, K=2, freq=6.0),
              dict(nx=21, nz=300, npml=4, K=2, freq=6.0)]
    gpus, rhs = [], []
    for q, sh in enumerate(shapes):
        print(f"[case] mixed-kernel FP64 batch member {q}: {sh}", flush=True)
        g = KKTProblem.from_inputs(tiny_inputs(seed=q, **sh), eps=1.0)
        g.set_solver_shape(3, 2)
        gpus.append(g)
        rhs.append(to_dev(complex_normal(g.field_shape, seed=50 + q)))
    singles = [g.helmholtz_solve(r, prec="c128", rtol=1e-30)[0] for g, r in zip(gpus, rhs)]
    batch = KKTBatch(gpus)
    xs = batch.helmholtz_solve(rhs, prec="c128")
    batch.close()
    for g, x, s1, r in zip(gpus, xs, singles, rhs):
        res = rel(to_np(g.stencil_apply(x)), to_np(r))
        print(f"member nz={g.nz}: batch vs single {rel(to_np(x), to_np(s1)):.1e}, residual {res:.1e}", flush=True)
        assert rel(to_np(x), to_np(s1)) <= 1e-12
        assert res <= 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_batch_with_uneven_chunk_counts_matches_single_problem_solves(prec):
    """Members cut into 1, 2, 5 and 8 chunks share one batch: no separators, a root
    alone, and reduction levels whose separators have two or three terms, each term's
    product in a workgroup of its own and the partials added per member."""
    shapes = [(dict(nx=21, nz=15, npml=4, K=3, freq=4.0), 1), (dict(nx=25, nz=19, npml=4, K=2, freq=6.0), 2),
              (dict(nx=41, nz=23, npml=4, K=5, freq=6.0), 5), (dict(nx=47, nz=17, npml=4, K=18, freq=8.0), 8)]
    dt = torch.complex64 if prec == "c64" else torch.complex128
    gpus, rhs = [], []
    for q, (sh, chunks) in enumerate(shapes):
        print(f"[case] uneven-chunk batch member {q}: {sh}, {chunks} chunks, {prec}", flush=True)
        g = KKTProblem.from_inputs(tiny_inputs(seed=q, **sh), eps=1.0)
        g.set_solver_shape(chunks, 2)
        gpus.append(g)
        rhs.append(to_dev(complex_normal(g.field_shape, seed=60 + q), dt))
    singles = [g.helmholtz_solve(r, prec=prec)[0] for g, r in zip(gpus, rhs)]
    batch = KKTBatch(gpus)
    xs = batch.helmholtz_solve(rhs, prec=prec)
    batch.close()
    for g, x, s1, r in zip(gpus, xs, singles, rhs):
        r64 = r.to(torch.complex128)
        res = rel(to_np(g.stencil_apply(x.to(torch.complex128))), to_np(r64))
        print(f"member nz={g.nz}: batch vs single {rel(to_np(x), to_np(s1)):.1e}, residual {res:.1e}", flush=True)
        assert rel(to_np(x), to_np(s1)) <= (1e-12 if prec == "c128" else 1e-5)
        assert res <= (1e-12 if prec == "c128" else 1e-4)
