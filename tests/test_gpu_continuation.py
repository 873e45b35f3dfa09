"""Frequency continuation on the GPU (newton_continuation, Section 6: frequencies from
low to high, each starting from the model the previous one reached, each with its own
eps) against the oracle's composition of exact Newton steps."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle.kkt import Problem, continuation  # noqa: E402
from paper_2204_06489_amd.solver import KKTProblem, newton_continuation  # noqa: E402
from tests.gpu_cases import eps_rule, rel, tiny_inputs, to_dev, to_np  # noqa: E402


def test_continuation_matches_oracle():
    inp = tiny_inputs(nx=41, nz=19, npml=4, K=3, weights="random")
    freqs, steps = (4.0, 6.0, 8.0), (2, 1, 2)
    print(f"[case] continuation 41x19 K=3 freqs {freqs} steps {steps}", flush=True)
    orc, gpu, data = [], [], []
    for f in freqs:
        q = dict(inp, freq=f, omega=2 * np.pi * f)
        pt = Problem.from_inputs(q, gamma=q["gamma_true"], eps=1.0)
        data.append(pt.sample(pt.forward()))
        p0 = Problem.from_inputs(q, eps=1.0, reg_on_update=True)
        eps = eps_rule(p0, p0.forward())          # each frequency's own eps (the ramp)
        orc.append(Problem.from_inputs(q, eps=eps, reg_on_update=True))
        gpu.append(KKTProblem.from_inputs(q, eps=eps, reg_on_update=True))
    g_ref, mis_ref = continuation(orc, data, steps)
    g, st = newton_continuation(gpu, [to_dev(d) for d in data], steps, rtol=1e-11, restart=30, maxit=200,
                                pc="exact")
    assert len(st) == sum(steps)
    mis = [s["misfit_before"] for s in st]
    print("misfits GPU", np.round(mis, 6), "oracle", np.round(mis_ref, 6))
    assert np.allclose(mis, mis_ref, rtol=1e-9)
    assert rel(to_np(g), g_ref) <= 1e-10
    assert torch.equal(gpu[-1].get_gamma(), g)


def test_continuation_rejects_mixed_grids():
    from paper_2204_06489_amd._lib import KF_ESHAPE, KFError
    a = KKTProblem.from_inputs(tiny_inputs(nx=41, nz=19, npml=4, K=3), eps=1.0)
    b = KKTProblem.from_inputs(tiny_inputs(nx=43, nz=19, npml=4, K=3), eps=1.0)
    d = torch.zeros((3, a.nrec), dtype=torch.complex128, device="cuda")
    db = torch.zeros((3, b.nrec), dtype=torch.complex128, device="cuda")
    with pytest.raises(KFError) as e:
        newton_continuation([a, b], [d, db], [1, 1])
    assert e.value.status == KF_ESHAPE
