"""kkt_apply_noalloc (the KKT matvec that allocates nothing: its source groups' parts of
the control row live in the library's file-scope device array) against kkt_apply, through
the C ABI, on two calls in a row: the 801 x 281, 80-source workload, then a smaller
133 x 37, 5-source problem (the array keeps the first call's contents)."""

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2204_06489_amd._lib import check, lib  # noqa: E402
from paper_2204_06489_amd.solver import KKTProblem  # noqa: E402
from synthetic import complex_normal, make_problem_inputs  # noqa: E402
from tests.oracle_cases import tiny_inputs  # noqa: E402


def _noalloc(p, xi):
    L = lib()
    fn = L.kkt_apply_noalloc
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    y = torch.full((p.Nxi,), float("nan"), dtype=torch.complex128, device="cuda")
    check(fn(p._h, C.c_void_p(xi.data_ptr()), C.c_void_p(y.data_ptr())))
    return y


def _case(inp, seed):
    p = KKTProblem.from_inputs(inp, eps=inp.get("eps") or 3.7e9)
    u = torch.as_tensor(complex_normal(p.field_shape, seed=seed)).cuda()
    p.set_background(u)
    xi = torch.as_tensor(complex_normal(p.Nxi, seed=seed + 1)).cuda()
    return p, xi


def test_noalloc_matches_kkt_apply_on_two_calls():
    big = make_problem_inputs("c2", 0)
    small = tiny_inputs(nx=133, nz=37, npml=6, K=5, nrec=7, weights="random")
    for name, inp, seed in (("801x281 K=80", big, 50), ("133x37 K=5", small, 60)):
        print(f"[case] kkt_apply_noalloc {name}", flush=True)
        p, xi = _case(inp, seed)
        ref = p.kkt_apply(xi)
        y = _noalloc(p, xi)
        torch.cuda.synchronize()
        ref_n, y_n = ref.cpu().numpy(), y.cpu().numpy()
        assert np.all(np.isfinite(y_n))
        err = np.linalg.norm(y_n - ref_n) / np.linalg.norm(ref_n)
        for a, b in zip(p.unpack(y), p.unpack(ref)):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
        print(f"{name}: relative difference {err:.1e}")
        p.close()
