"""Block solves whose columns take each kind of sweep kernel at ragged heights.

Columns of up to 144 rows take the matrix-core sweeps with three wavefronts, up to 288
rows with six (a column height just past 144 leaves most of the last row tiles empty),
taller ones the vector units; the spikes of the factorisation follow the same split.
Each height is solved with three chunks (so the spikes, the separators' reduction and
the interior correction all run) and 21 sources (a full and a ragged 16-source tile),
forward and adjoint, in FP64, complex64 and the mixed refinement, against the FP64
oracle's banded LU."""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from synthetic import complex_normal  # noqa: E402
from tests.gpu_cases import oracle_and_gpu, rel, tiny_inputs, to_dev, to_np  # noqa: E402


@pytest.mark.parametrize("nz", [145, 203, 288, 289])
def test_tall_column_solves_match_banded_lu(nz):
    shape = dict(nx=23, nz=nz, npml=4, K=21)
    print(f"[case] tall columns {shape}, 3 chunks", flush=True)
    inp = tiny_inputs(seed=4, **shape)
    orc, gpu = oracle_and_gpu(inp, eps=1.0)
    gpu.set_solver_shape(3, 2)
    b = complex_normal(gpu.field_shape, seed=11)
    for adjoint in (False, True):
        ref = orc.lu.solve(b, adjoint=adjoint)
        x, st = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="c128", rtol=1e-30)
        err = rel(to_np(x), ref)
        print(f"  adjoint={adjoint} c128 error {err:.2e} residual {st['rel_res_max']:.2e}", flush=True)
        assert err <= 1e-10 and st["rel_res_max"] <= 1e-12
        x32, st32 = gpu.helmholtz_solve(to_dev(b, torch.complex64), adjoint=adjoint, prec="c64", rtol=1e-30)
        print(f"  adjoint={adjoint} c64 error {rel(to_np(x32), ref):.2e} residual {st32['rel_res_max']:.2e}",
              flush=True)
        assert st32["rel_res_max"] <= 1e-4
        assert rel(to_np(x32), ref) <= 1e-3
        xm, stm = gpu.helmholtz_solve(to_dev(b), adjoint=adjoint, prec="mixed", rtol=1e-11, maxit=10)
        assert stm["converged"] and rel(to_np(xm), ref) <= 1e-9
