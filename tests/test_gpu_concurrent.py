"""Newton steps of independent problems at once (newton_step_concurrent: a stream and a
host thread per problem, e.g. one problem per frequency on its own grid).  Every
problem must compute exactly what it computes alone (its kernels and their order on
its own stream are those of newton_step), the oracle's step included."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd.solver import KKTProblem, newton_step_concurrent  # noqa: E402
from tests.gpu_cases import eps_rule, observed_data, oracle_and_gpu, rel, to_dev, to_np  # noqa: E402
from tests.oracle_cases import tiny_inputs  # noqa: E402

SHAPES = [dict(nx=21, nz=15, npml=4, K=3, freq=4.0), dict(nx=41, nz=19, npml=4, K=2, freq=6.0),
          dict(nx=67, nz=37, npml=5, K=4, freq=8.0)]


def _problems(pc):
    ins = [tiny_inputs(seed=q, weights="random", **sh) for q, sh in enumerate(SHAPES)]
    data, orcs, gpus = [], [], []
    for q, inp in enumerate(ins):
        print(f"[case] concurrent member {q}: {SHAPES[q]}, {pc}", flush=True)
        d = observed_data(inp)
        orc, _ = oracle_and_gpu(inp, eps=1.0)
        eps = eps_rule(orc, orc.forward())
        orc, gpu = oracle_and_gpu(inp, eps=eps)
        data.append(d)
        orcs.append(orc)
        gpus.append(gpu)
    return ins, data, orcs, gpus


@pytest.mark.parametrize("pc", ["exact", "inexact"])
def test_concurrent_steps_equal_single_steps_and_the_oracle(pc):
    ins, data, orcs, gpus = _problems(pc)
    kw = dict(rtol=1e-10, restart=30, maxit=300, pc=pc, update_in_place=False)
    dd = [to_dev(d) for d in data]
    xis, gs, sts = newton_step_concurrent(gpus, dd, **kw)
    for q, (g, orc, d) in enumerate(zip(gpus, orcs, data)):
        xi1, g1, st1 = g.newton_step(dd[q], **kw)
        print(f"member {q}: iterations {sts[q]['outer_iters']} / {st1['outer_iters']}, "
              f"rel res {sts[q]['rel_res']:.2e}", flush=True)
        assert sts[q]["converged"] and sts[q]["outer_iters"] == st1["outer_iters"]
        assert torch.equal(xis[q], xi1) and torch.equal(gs[q], g1)
        u_n = orc.forward()
        ds_ref = orc.unpack(orc.kkt_solve_schur(u_n, orc.residual(d, u_n)))[1]
        assert rel(orc.unpack(to_np(xis[q]))[1], ds_ref) <= 1e-7


def test_concurrent_steps_report_maxit_and_give_the_streams_back():
    ins, data, orcs, gpus = _problems("exact")
    dd = [to_dev(d) for d in data]
    _, _, sts = newton_step_concurrent(gpus, dd, rtol=1e-12, restart=5, maxit=1, pc="exact", update_in_place=False,
                                       want_xi=False)
    assert all(not s["converged"] and s["outer_iters"] == 1 for s in sts)
    # the problems are back on their own streams: a plain step afterwards converges as before
    _, _, st = gpus[0].newton_step(dd[0], rtol=1e-10, restart=30, maxit=300, pc="exact", update_in_place=False)
    assert st["converged"]
    with pytest.raises(Exception, match="appears twice"):
        newton_step_concurrent([gpus[0], gpus[0]], [dd[0], dd[0]])


def test_concurrent_steps_report_the_first_failing_problem():
    ins, data, orcs, gpus = _problems("exact")
    dd = [to_dev(d) for d in data]
    print("[case] concurrent steps with an invalid restart length", flush=True)
    with pytest.raises(Exception, match="problem 0: .*restart"):
        newton_step_concurrent(gpus, dd, restart=0)
    # nothing was changed: the problems still step normally, alone and together
    _, gs, sts = newton_step_concurrent(gpus, dd, rtol=1e-10, restart=30, maxit=300, pc="exact",
                                        update_in_place=False, want_xi=False)
    assert all(s["converged"] for s in sts)
    assert all(torch.isfinite(g).all() for g in gs)
