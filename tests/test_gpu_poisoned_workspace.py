"""Every solver path on device buffers that start as NaN.

With KF_POISON_ALLOC set, the library fills each buffer it allocates with 0xFF bytes
(NaN in FP32 and FP64).  A kernel that reads an entry no kernel has written, even to
multiply it by zero, then turns the result into NaN, whatever the memory held before;
without the poison such a read depends on the allocator's history (fresh memory is
zero, reused memory holds the previous owner's values).  Each path is checked against
the oracle's exact step, so that a poisoned run is also a parity run.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_cases import oracle_and_gpu, observed_data, eps_rule, rel, tiny_inputs, to_dev, to_np  # noqa: E402

SHAPE = dict(nx=81, nz=37, npml=6, K=5, weights="random")


@pytest.fixture
def poisoned(monkeypatch):
    monkeypatch.setenv("KF_POISON_ALLOC", "1")
    inp = tiny_inputs(**SHAPE)
    d = observed_data(inp)
    orc, _ = oracle_and_gpu(inp, eps=1.0)
    u_n = orc.forward()
    eps = eps_rule(orc, u_n)
    orc, gpu = oracle_and_gpu(inp, eps=eps)
    return inp, orc, gpu, d, u_n


@pytest.mark.parametrize("chunks,ns", [(1, 1), (6, 2)])
def test_block_solves_on_poisoned_buffers(poisoned, chunks, ns):
    inp, orc, gpu, _, _ = poisoned
    print(f"[case] poisoned block solves 81x37 K=5, shape ({chunks}, {ns})", flush=True)
    gpu.set_solver_shape(chunks, ns)
    f = gpu.sources()
    ref = orc.forward()
    for prec, bar in (("c128", 1e-11), ("c64", 1e-4)):
        ff = f if prec == "c128" else f.to(torch.complex64)
        for adj in (False, True):
            x, _ = gpu.helmholtz_solve(ff, adjoint=adj, prec=prec)
            x = to_np(x).astype(np.complex128)
            assert np.isfinite(x).all(), (prec, adj)
            if not adj:
                assert rel(x, ref) <= bar, prec


@pytest.mark.parametrize("form", ["fgmres-exact", "fgmres-inexact-mixed", "bicgstab-inexact", "rsgn"])
def test_newton_forms_on_poisoned_buffers(poisoned, form):
    inp, orc, gpu, d, u_n = poisoned
    print(f"[case] poisoned Newton step 81x37 K=5, {form}", flush=True)
    gpu.set_solver_shape(6, 2)
    xi_ref = orc.kkt_solve_schur(u_n, orc.residual(d, u_n))
    ds_ref = orc.unpack(xi_ref)[1]
    dd = to_dev(d)
    if form == "rsgn":
        ds, _, st = gpu.rsgn_step(dd, rtol=1e-11, maxit=500, update_in_place=False)
        assert st["converged"]
        assert rel(to_np(ds), ds_ref) <= 1e-8
        return
    kw = {"fgmres-exact": dict(pc="exact"),
          "fgmres-inexact-mixed": dict(pc="inexact", fwd_prec="mixed"),
          "bicgstab-inexact": dict(pc="inexact", outer="bicgstab")}[form]
    xi, g1, st = gpu.newton_step(dd, rtol=1e-10, maxit=400, update_in_place=False, **kw)
    assert st["converged"] and st["rel_res"] <= 1e-10
    assert rel(orc.unpack(to_np(xi))[1], ds_ref) <= 1e-7
    assert rel(to_np(g1), orc.update(ds_ref)) <= 1e-9


def test_multigrid_on_poisoned_buffers(poisoned):
    inp, orc, gpu, _, _ = poisoned
    print("[case] poisoned multigrid solve 81x37 K=5", flush=True)
    gpu.set_multigrid(prec="c128", inner_rtol=1e-3, n_min=8)
    f = gpu.sources()
    x, st = gpu.helmholtz_solve_mg(f, rtol=1e-8, maxit=300)
    assert st["converged"] and st["levels"] >= 2
    assert rel(to_np(x), orc.forward()) <= 1e-6
