"""Write the FP64 oracle's Newton step on one of the timed workloads.

Calls only the oracle (banded-LU forward solves, assembled KKT matrix, right-
preconditioned GMRES with the exact banded-LU preconditioner of eq. precond) and
stores what the mixed-precision GPU step is compared with: ds, gamma_{n+1}, the
misfit before and after the step, and the KKT relative residual reached.

Usage: python -m tests.golden.make_newton_reference CONFIG FREQ_INDEX OUT.npz [TOL]
  c2 0 tests/golden/c2_newton_oracle.npz 1e-10   801 x 281, 80 sources, 5 Hz (about an hour of CPU)
  c1 1 tests/golden/c1_newton_oracle.npz 1e-12   401 x 141, 40 sources, 5 Hz (several minutes)
TOL is the GMRES relative residual target (default 1e-12, near the FP64 floor of
these systems, so that the stored step is the exact KKT solution to ~1e-12).
"""

import sys
import time

import numpy as np

from oracle.kkt import Problem, gmres_right
from synthetic.configs import make_problem_inputs



def main(config, freq_index, out, tol=1e-12):
    t0 = time.time()
    inp = make_problem_inputs(config, freq_index)
    pt = Problem.from_inputs(inp, gamma=inp["gamma_true"], eps=inp["eps"])
    d = pt.sample(pt.forward())
    del pt
    print(f"data ({time.time() - t0:.0f}s)", flush=True)
    p = Problem.from_inputs(inp, eps=inp["eps"], reg_on_update=True)
    u_n = p.forward()
    r = p.residual(d, u_n)
    b = p.rhs(r)
    M = p.assemble_M(u_n)
    print(f"setup ({time.time() - t0:.0f}s)", flush=True)
    it = [0]

    def apply_M(v):
        return M @ v

    def apply_P(v):
        it[0] += 1
        if it[0] % 5 == 0:
            print(f"  precond {it[0]} ({time.time() - t0:.0f}s)", flush=True)
        return p.precond_apply(u_n, v)

    xi, hist, _ = gmres_right(apply_M, apply_P, b, tol=tol, restart=15, maxit=600)
    rel = np.linalg.norm(b - M @ xi) / np.linalg.norm(b)
    ds = p.unpack(xi)[1]
    g1 = p.update(ds)
    q = Problem.from_inputs(inp, gamma=g1, eps=inp["eps"])
    u1 = q.forward()
    mis0 = np.linalg.norm(r) / np.linalg.norm(d)
    mis1 = np.linalg.norm(d - q.sample(u1)) / np.linalg.norm(d)
    np.savez_compressed(out, ds=ds, gamma_next=g1, misfit_before=mis0, misfit_after=mis1, rel_res=rel,
                        iterations=len(hist) - 1, d=d, tol=tol)
    print(f"done: {len(hist) - 1} iterations rel_res={rel:.2e} misfit {mis0:.4e} -> {mis1:.4e} "
          f"({time.time() - t0:.0f}s)", flush=True)


if __name__ == "__main__":
    if len(sys.argv) not in (4, 5):
        sys.exit(__doc__)
    main(sys.argv[1], int(sys.argv[2]), sys.argv[3], *(float(a) for a in sys.argv[4:]))
