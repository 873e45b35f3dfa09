"""Write the regularisation weights eps of every workload into synthetic/eps_table.json.

The paper leaves eps unspecified for the single-step experiment and gives an
unitless 10 -> 1e5 ramp for the frequency sweep (Section 6).  Its Hessian
H = J^* W^T W J + eps I is positive definite for any eps > 0 (Section 3); the
rule taken here is eps = 1e-2 * lambda_max(sum_k J_k^* W_k^2 J_k) at the initial
model, which bounds cond(H) by 101.  lambda_max comes from seeded power
iteration with this oracle; the result is an input literal shared by the
oracle and the GPU path.

Usage:  python -m oracle.make_eps c0 c1 [c2 c4]
"""

import json
import sys
import time

import numpy as np

from synthetic.configs import CONFIGS, EPS_TABLE_PATH, make_problem_inputs
from oracle.kkt import Problem

REL = 1e-2


def lambda_max(apply, n, iters, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply(v)
        lam = float(np.real(np.vdot(v, w)))
        v = w / np.linalg.norm(w)
    return lam


def main(names):
    try:
        with open(EPS_TABLE_PATH) as fh:
            table = json.load(fh)
    except FileNotFoundError:
        table = {}
    for name in names:
        cfg = CONFIGS[name]
        iters = 20 if name in ("c0", "c1", "c3") else 8
        for fi, f in enumerate(cfg["freqs"]):
            gi = fi if len(cfg["grids"]) > 1 else 0
            t0 = time.time()
            inp = make_problem_inputs(name, fi, gi)
            p = Problem.from_inputs(inp, eps=1.0)
            u_n = p.forward()
            lam = lambda_max(p.gn_operator(u_n), p.Ng, iters)
            table[f"{name}/g{gi}/{f:g}"] = REL * lam
            print(f"{name} grid {gi} f={f:g} Hz: lambda_max={lam:.6e} eps={REL * lam:.6e} "
                  f"({time.time() - t0:.1f}s)", flush=True)
            with open(EPS_TABLE_PATH, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c0", "c1"])
