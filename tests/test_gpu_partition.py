"""GPU tests of the partitioned block solver: every chunk count (down to one-column
chunks) and every source grouping solves A x = b and A^H x = b to the FP64 oracle's
banded LU within 1e-10, and the shapes agree with each other to rounding."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd._lib import KFError  # noqa: E402
from synthetic import complex_normal  # noqa: E402
from tests.gpu_cases import oracle_and_gpu, rel, tiny_inputs, to_dev, to_np  # noqa: E402

SHAPE = dict(nx=67, nz=37, npml=5, K=5)


@pytest.mark.parametrize("chunks", [1, 2, 3, 7, 16, 34])
@pytest.mark.parametrize("ns", [1, 2, 4, 8])
def test_partitioned_solve_matches_banded_lu(chunks, ns):
    print(f"[case] partition chunks={chunks} ns={ns} {SHAPE}", flush=True)
    inp = tiny_inputs(seed=1, **SHAPE)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    gpu.set_solver_shape(chunks, ns)
    assert gpu.solver_shape == (chunks, ns)
    b = complex_normal(gpu.field_shape, seed=7)
    for adjoint in (False, True):
        ref = orc.lu.solve(b, adjoint=adjoint)
        x, st = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="c128", rtol=1e-30)
        err = rel(to_np(x), ref)
        print(f"  adjoint={adjoint} c128 error {err:.2e} residual {st['rel_res_max']:.2e}")
        assert err <= 1e-10 and st["rel_res_max"] <= 1e-12
        x32, st32 = gpu.helmholtz_solve(to_dev(b, torch.complex64), adjoint=adjoint, prec="c64", rtol=1e-30)
        assert st32["rel_res_max"] <= 1e-4
        assert rel(to_np(x32), ref) <= 1e-3
        xm, stm = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="mixed", rtol=1e-11, maxit=10)
        assert stm["converged"] and rel(to_np(xm), ref) <= 1e-9


def test_shapes_agree_and_reshape_refactors():
    inp = tiny_inputs(seed=2, nx=133, nz=37, npml=6, K=3)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    b = to_dev(complex_normal(gpu.field_shape, seed=9))
    xs = []
    for chunks, ns in [(1, 1), (8, 2), (0, 0), (64, 4), (5, 1)]:
        gpu.set_solver_shape(chunks, ns)
        xs.append(to_np(gpu.helmholtz_solve(b, prec="c128")[0]))
    for x in xs[1:]:
        assert rel(x, xs[0]) <= 1e-11
    assert rel(xs[0], orc.lu.solve(to_np(b))) <= 1e-10


def test_invalid_shapes_are_rejected():
    inp = tiny_inputs(seed=0, nx=21, nz=15, npml=4, K=2)
    _, gpu = oracle_and_gpu(inp, eps=1.0)
    for chunks, ns in [(-1, 1), (12, 1), (65, 1), (2, 3), (2, 16)]:
        with pytest.raises(KFError):
            gpu.set_solver_shape(chunks, ns)
    gpu.set_solver_shape(11, 4)    # (nx + 1) / 2 one-column chunks
    assert gpu.solver_shape == (11, 4)


def test_autotune_picks_a_best_measured_shape_and_stays_exact():
    """The chosen shape is the best measured one, or (when a count refined around the
    coarse grid's best scored better by at most 2%) the coarse grid's best."""
    inp = tiny_inputs(seed=3, nx=133, nz=37, npml=6, K=9)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    table = gpu.autotune(prec="c64", solves_per_factor=50.0)
    print("autotune table (best first):", table[:4], "chosen:", gpu.solver_shape)
    assert len(table) >= 4
    for r in table:
        assert r["t_factor_ms"] > 0 and r["t_solve_ms"] > 0
        assert abs(r["score_ms"] - (r["t_factor_ms"] + 50.0 * r["t_solve_ms"])) <= 1e-9 * r["score_ms"]
    chosen = [r for r in table if (r["chunks"], r["sources_per_group"]) == gpu.solver_shape]
    assert len(chosen) == 1
    assert chosen[0]["score_ms"] * 0.98 <= table[0]["score_ms"] * (1 + 1e-12)
    b = complex_normal(gpu.field_shape, seed=4)
    x, _ = gpu.helmholtz_solve(to_dev(b), prec="c128")
    assert rel(to_np(x), orc.lu.solve(b)) <= 1e-10
    # a new problem of the same size starts from the tuned shape
    _, gpu2 = oracle_and_gpu(inp, eps=1.0)
    assert gpu2.solver_shape == gpu.solver_shape


def test_profiling_records_the_selected_family_only():
    inp = tiny_inputs(seed=2, **SHAPE)
    _, gpu = oracle_and_gpu(inp, eps=1.0)
    gpu.set_solver_shape(7, 1)
    b = to_dev(complex_normal(gpu.field_shape, seed=9), torch.complex64)
    gpu.profile_enable(True)
    gpu.profile_only("blu_correct")
    gpu.helmholtz_solve(b, prec="c64")
    assert gpu.profile_read("blu_correct")[0] == 1
    assert gpu.profile_read("blu_fwd_c64")[0] == 0
    gpu.profile_only(None)
    gpu.helmholtz_solve(b, prec="c64")
    assert gpu.profile_read("blu_correct")[0] == 2
    assert gpu.profile_read("blu_fwd_c64")[0] == 1
    with pytest.raises(KFError):
        gpu.profile_only("no_such_family")
    gpu.profile_enable(False)
