#!/usr/bin/env python3
"""Benchmark: full-space Gauss-Newton step time on one MI355X (and KKT-matvec GB/s).

One step = one whole Newton step of the method on the GPU (Sections 3-5): block
factorisation of A(gamma_n), background solve u_n = A^-1 f, data residual and
KKT right-hand side, flexible GMRES with the block-triangular preconditioner to
||b - M xi|| <= 1e-6 ||b||, and the update gamma_{n+1} = gamma_n + Re(ds), which
the next step continues from.

Workload (default): the 401 x 141 grid (h = 10 m, 20-cell PML) of the seeded
faulted-lens earth, 40 sources and 401 receivers on the first core row, 5 Hz,
inexact preconditioner (complex64 block sweeps), FGMRES(30), b_s = 0.  Inputs
are synthetic; the observed data are a forward solve of the true model.

Prints one JSON line.  Also reported:
  roofline      the kernel with the most GPU time in the timed steps, timed live
                with HIP events on the library's stream;
  kkt_apply     the fused KKT matvec at this size and at 801 x 281 x 80 sources
                (1.45 GB per call, larger than the 256 MB Infinity Cache);
  cpu_baseline  the FP64 oracle (banded LU, the paper's own CPU algorithm) timed on
                a bounded sample of the same workload on the host.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--freq-index", type=int, default=1)
    ap.add_argument("--pc", default="inexact", choices=["exact", "inexact"])
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-kkt", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the automatic solver shape")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain device copy of 1 GiB (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def partition(nx, chunks):
    """Chunks of the partitioned block solver: (first, last, meeting column) per chunk,
    interior lengths as even as possible around chunks - 1 separator columns (the
    library's own rule, repeated here to count the work)."""
    n_int = nx - (chunks - 1)
    base, extra = divmod(n_int, chunks)
    out, a = [], 0
    for c in range(chunks):
        L = base + (1 if c < extra else 0)
        out.append((a, a + L - 1, a + L // 2))
        a += L + 1
    return out


def kernel_work(name, p):
    """Algorithmic work of one launch of a kernel family: (amount, unit, dtype)."""
    nx, nz, K, Nu, Ng = p.nx, p.nz, p.K, p.Nu, p.Ng
    m = nz
    P = p.solver_shape[0]
    part = partition(nx, P)
    if name == "kkt_apply":
        # read du, lambda, u_n, write y_u, y_lambda per node-source; gamma per node;
        # ds read + y_s write per control node (receiver term is a separate kernel)
        return Nu * (80 * K + 8) + 32 * Ng, "bytes", "f64"
    if name == "blu_factor":
        # one m x m complex inversion per column (m^3 complex multiply-adds, 8 flops each),
        # the spikes (a chunk solve with m right-hand sides: forward over the loaded half,
        # the middle, back-substitution over the other columns), and the separator
        # system by block cyclic reduction (an inversion per separator, and per level
        # F, G for the eliminated separators and up to six products for the others)
        inv = nx
        spike = sum((mid - a if w == 0 else b - mid) + (b - a + 1)
                    for c, (a, b, mid) in enumerate(part) for w in (0, 1)
                    if (w == 0 and c > 0) or (w == 1 and c < P - 1))
        red, n = 0, P - 1
        st = 1
        while 2 * st <= n:
            red += sum((j - st >= 1) + (j + st <= n) for j in range(st, n + 1, 2 * st))
            red += sum(2 + (k - 2 * st >= 1) + 2 * (k + st <= n) + (k + 2 * st <= n) for k in range(2 * st, n + 1, 2 * st))
            st *= 2
        return 8.0 * m ** 3 * (inv + spike + red), "flops", "f64"
    dt = "f32" if name.endswith("c64") or name == "blu_correct" else "f64"
    if name.startswith("blu_fwd") or name.startswith("blu_bwd"):
        # a dense m x m complex matvec per column and source: every chunk column but the middle
        cols = sum(b - a for a, b, mid in part)
        return 8.0 * m * m * cols * K, "flops", dt
    if name == "blu_correct":
        # V_i and / or W_i (m x m) times the separator values, every interior column and source
        blocks = sum((b - a + 1) * ((1 if c > 0 else 0) + (1 if c < P - 1 else 0)) for c, (a, b, mid) in enumerate(part))
        return 8.0 * m * m * blocks * K, "flops", dt
    raise KeyError(name)


MFMA_KERNELS = ("blu_fwd_c64", "blu_bwd_c64", "blu_correct")


def roofline_for(name, p, launches, total_ms):
    amount, unit, dt = kernel_work(name, p)
    avg_s = total_ms / launches * 1e-3
    if unit == "bytes":
        achieved = amount / avg_s / 1e9
        peak = HBM_PEAK_GBS
        out = {"bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s"}
    else:
        achieved = amount / avg_s / 1e12
        peak = FP32_PEAK_TFLOPS if dt == "f32" else FP64_PEAK_TFLOPS
        # complex64 sweeps and the interior correction run on the matrix cores (dense
        # FP32 MFMA peak); the FP64 sweeps on the vector units (FP64 vector peak)
        # (the matrix-core sweeps take columns of up to 288 rows)
        bound = "mfma" if name == "blu_correct" or (name in MFMA_KERNELS and p.nz <= 288) else "alu"
        out = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    out.update({"frac": achieved / peak, "traffic": None, "kernel": name, "launches": launches,
                "avg_launch_us": total_ms / launches * 1e3, "work_per_launch": amount, "work_unit": unit})
    return out


def measured_traffic(name, config):
    """HBM bytes per launch from the committed rocprofv3 counter runs (taken on the
    401x141, 40-source workload, c1), or None for another workload or once the kernel
    sources differ from the build the counters were taken on."""
    if config != "c1":
        return None
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    tab = json.load(open(path))
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2204_06489_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    k = tab.get("kernels", {}).get(name)
    if k is None or h.hexdigest()[:16] != tab.get("source_sha"):
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def observed_data(inp, torch, KKTProblem):
    pt = KKTProblem.from_inputs(inp, gamma=inp["gamma_true"])
    u, _ = pt.helmholtz_solve(pt.sources())
    riz = torch.as_tensor(inp["rec_iz"]).long().cuda()
    rix = torch.as_tensor(inp["rec_ix"]).long().cuda()
    d = u[:, riz, rix].contiguous()
    del u
    pt.close()
    return d


def hbm_kkt(torch, KKTProblem, args):
    """kkt_apply at 801 x 281, 80 sources (working set far above the Infinity Cache)."""
    from synthetic.configs import make_problem_inputs
    inp = make_problem_inputs("c2", 0)
    p = KKTProblem.from_inputs(inp, eps=inp["eps"] or 1.0)
    g = torch.Generator(device="cuda").manual_seed(1234)
    u = torch.randn(p.field_shape, dtype=torch.complex128, device="cuda", generator=g)
    p.set_background(u)
    xi = torch.randn(p.Nxi, dtype=torch.complex128, device="cuda", generator=g)
    y = p.empty_xi()
    for _ in range(3):
        p.kkt_apply(xi, out=y)
    torch.cuda.synchronize()
    p.profile_enable(True)
    for _ in range(20):
        p.kkt_apply(xi, out=y)
    n, ms = p.profile_read("kkt_apply")
    p.profile_enable(False)
    r = roofline_for("kkt_apply", p, n, ms)
    p.close()
    del u, xi, y
    # a plain 1 GiB device-to-device copy on torch's stream: the streaming rate this
    # machine reaches for a read + write mix, next to the published HBM peak
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return {"grid": "801x281", "K": 80, "GB_per_call": r["work_per_launch"] / 1e9,
            "avg_launch_us": r["avg_launch_us"], "GB_s": r["achieved"], "frac_of_hbm_peak": r["frac"],
            "copy_GB_s": copy_gbs, "frac_of_copy": r["achieved"] / copy_gbs}


def cpu_baseline(inp, gpu_iters, args):
    """The oracle (numpy/scipy, banded LU) on a bounded sample of the same step."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.kkt import Problem, gmres_right
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        p = Problem.from_inputs(inp, gamma=inp["gamma0"], eps=inp["eps"], reg_on_update=True)
        t_factor = time.perf_counter() - t0
        t0 = time.perf_counter()
        u_n = p.forward()
        t_fwd = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        d = p.sample(u_n) * (1.0 + 0.1 * rng.standard_normal((p.K, p.nrec)))
        b = p.rhs(p.residual(d, u_n))
        n_it = 2
        t0 = time.perf_counter()
        gmres_right(lambda v: p.kkt_apply(u_n, v), lambda v: p.precond_apply(u_n, v), b, tol=1e-30,
                    restart=args.restart, maxit=n_it)
        t_it = (time.perf_counter() - t0) / n_it
    est = t_factor + t_fwd + gpu_iters * t_it
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"full-size banded-LU factorisation ({t_factor:.1f} s), background solve ({t_fwd:.1f} s) "
                       f"and {n_it} right-preconditioned GMRES iterations with the exact banded-LU "
                       f"preconditioner ({t_it:.1f} s each), scaled to the GPU step's {gpu_iters:.1f} outer "
                       f"iterations; one BLAS thread")}


def bench_c4(args, torch, KKTProblem):
    """Five frequencies (2-10 Hz) on five grids (201x71 ... 1001x351), 100 sources each:
    one batched Newton step for all of them (persistent launches, hipGraph columns),
    and the same five problems stepped one after another for comparison."""
    import numpy as np
    from synthetic.configs import make_problem_inputs
    from paper_2204_06489_amd.solver import KKTBatch
    inps = [make_problem_inputs("c4", fi) for fi in range(5)]
    probs, ds = [], []
    for inp in inps:
        log(args, f"c4 problem {inp['nx']}x{inp['nz']} f={inp['freq']:g} Hz K={inp['K']}")
        ds.append(observed_data(inp, torch, KKTProblem))
        probs.append(KKTProblem.from_inputs(inp, reg_on_update=True))
        if not args.no_autotune:
            best = probs[-1].autotune(prec="c64" if args.pc == "inexact" else "c128", solves_per_factor=100.0)[0]
            log(args, f"  autotuned shape P={best['chunks']} ns={best['sources_per_group']}")
    g0 = [torch.as_tensor(inp["gamma0"]).cuda() for inp in inps]

    def reset():
        # every timed pass starts from gamma_0, so both passes factorise and solve the same systems
        for p, g in zip(probs, g0):
            p.set_gamma(g)
        torch.cuda.synchronize()

    batch = KKTBatch(probs)
    kw = dict(rtol=args.rtol, restart=20, maxit=600, pc=args.pc, update_in_place=True, want_xi=False)
    for w in range(args.warmup):
        batch.newton_step(ds, use_graph=True, **kw)
    reset()
    t0 = time.perf_counter()
    sts = []
    for k in range(args.steps):
        _, _, st = batch.newton_step(ds, use_graph=True, **kw)
        sts.append(st)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    for k, st in enumerate(sts):
        log(args, f"batched step {k}: iters {[s['outer_iters'] for s in st]} factor {st[0]['t_factor_ms']:.0f} ms "
                  f"fwd {st[0]['t_forward_ms']:.0f} ms columns {st[0]['t_precond_ms']:.0f} ms "
                  f"orth {st[0]['t_orth_ms']:.0f} ms total {st[0]['t_total_ms']:.0f} ms")
    # the same batch with every launch enqueued directly (no graph replay)
    reset()
    t0 = time.perf_counter()
    for k in range(args.steps):
        batch.newton_step(ds, use_graph=False, **kw)
    torch.cuda.synchronize()
    t_batch_nograph = (time.perf_counter() - t0) / args.steps
    log(args, f"batched without graphs: {t_batch_nograph * 1e3:.0f} ms per step")
    batch.close()
    # the same problems one at a time, each from gamma_0 again
    reset()
    t0 = time.perf_counter()
    seq = []
    for k in range(args.steps):
        for p, d in zip(probs, ds):
            _, _, st = p.newton_step(d, rtol=args.rtol, restart=20, maxit=600, pc=args.pc, fwd_prec="c128",
                                     update_in_place=True, want_xi=False)
            seq.append(st)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.steps
    log(args, f"one at a time: {t_seq*1e3:.0f} ms per step, iters {[s['outer_iters'] for s in seq]}, "
              f"factor {[round(s['t_factor_ms']) for s in seq]} ms, total {[round(s['t_total_ms']) for s in seq]} ms, "
              f"precond {[round(s['t_precond_ms']) for s in seq]} ms, matvec {[round(s['t_matvec_ms']) for s in seq]} ms, "
              f"orth {[round(s['t_orth_ms']) for s in seq]} ms")
    # the two smallest grids alone, where neither fills the chip: batched against one at a time
    small = KKTBatch(probs[:2])
    small.newton_step(ds[:2], use_graph=True, **kw)
    reset()
    t0 = time.perf_counter()
    for k in range(args.steps):
        small.newton_step(ds[:2], use_graph=True, **kw)
    torch.cuda.synchronize()
    t_small_batch = (time.perf_counter() - t0) / args.steps
    small.close()
    reset()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for p, d in zip(probs[:2], ds[:2]):
            p.newton_step(d, rtol=args.rtol, restart=20, maxit=600, pc=args.pc, fwd_prec="c128",
                          update_in_place=True, want_xi=False)
    torch.cuda.synchronize()
    t_small_seq = (time.perf_counter() - t0) / args.steps
    log(args, f"201x71 + 401x141 only: batched {t_small_batch*1e3:.0f} ms, one at a time {t_small_seq*1e3:.0f} ms per step")
    result = {
        "metric": "Newton-step time to KKT rel. res 1e-6", "value": t_batch, "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c128 outer (FP64) + c64 block sweeps" if args.pc == "inexact" else "c128",
        "data": "synthetic",
        "config": {"workload": ("c4: one Newton step at 2, 4, 6, 8 and 10 Hz on the 201x71, 401x141, 601x211, "
                                "801x281 and 1001x351 grids (20-cell PML), 100 sources each, batched: "
                                "persistent work-list launches for every factorisation and block solve, "
                                "hipGraph replay of each FGMRES column, FGMRES(20) to " + f"{args.rtol:g}"),
                   "global_batch": 500, "parallelism": "single GPU"},
        "one_at_a_time_s": t_seq,
        "batched_without_graphs_s": t_batch_nograph,
        "two_smallest_grids": {"grids": ["201x71", "401x141"], "batched_s": t_small_batch,
                               "one_at_a_time_s": t_small_seq},
        "per_problem": [{"grid": f"{i['nx']}x{i['nz']}", "freq": i["freq"], "iters": s["outer_iters"],
                         "rel_res": s["rel_res"], "misfit": s["misfit_before"]} for i, s in zip(inps, sts[-1])],
    }
    print(json.dumps(result), flush=True)


def bench_c3(args, torch, KKTProblem):
    """Reduced gradient through the solve at 801 x 281, 80 sources, 5 Hz: autograd
    forward (factorisation + forward solves) and backward (adjoint solves + gradient
    kernel), complex128 and complex64.  Each step perturbs gamma, so it refactorises."""
    from synthetic.configs import make_problem_inputs
    from paper_2204_06489_amd.autograd import HelmholtzSolve
    inp = make_problem_inputs("c2", 0)
    log(args, f"c3 timing on {inp['nx']}x{inp['nz']} K={inp['K']} {inp['freq']} Hz")
    d = observed_data(inp, torch, KKTProblem)
    p = KKTProblem.from_inputs(inp, reg_on_update=True)
    g0 = torch.as_tensor(inp["gamma0"]).cuda()
    riz = torch.as_tensor(inp["rec_iz"]).long().cuda()
    rix = torch.as_tensor(inp["rec_ix"]).long().cuda()
    res = {}
    for prec in ("c128", "c64"):
        def step(k):
            x = (g0 * (1.0 + 1e-4 * k)).requires_grad_(True)
            u = HelmholtzSolve.apply(x, p, prec)
            loss = 0.5 * torch.sum(torch.abs(d.to(u.dtype) - u[:, riz, rix]) ** 2)
            loss.backward()
            return x.grad
        for w in range(args.warmup):
            step(w + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(100 + k)
        torch.cuda.synchronize()
        res[prec] = (time.perf_counter() - t0) / args.steps
        log(args, f"{prec}: {res[prec] * 1e3:.1f} ms per gradient")
    result = {
        "metric": "reduced-gradient time (autograd forward + backward)", "value": res["c64"], "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["c64"] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "c3: torch.autograd.Function around the batched Helmholtz solve on the 801x281 grid, "
                               "80 sources, 5 Hz; one step = factorisation, forward solves, misfit, adjoint solves "
                               "and the gradient kernel", "global_batch": inp["K"], "parallelism": "single GPU"},
        "c128_s": res["c128"],
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU source sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from synthetic.configs import make_problem_inputs
    from paper_2204_06489_amd.solver import KKTProblem

    torch.cuda.set_device(0)
    if args.config == "c4":
        return bench_c4(args, torch, KKTProblem)
    if args.config == "c3":
        return bench_c3(args, torch, KKTProblem)
    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": a.numel() * 8, "launches": 3}))
        return
    inp = make_problem_inputs(args.config, args.freq_index)
    if inp["eps"] is None:
        raise SystemExit("no eps for this workload in synthetic/eps_table.json")
    log(args, f"workload {args.config} f={inp['freq']} Hz grid {inp['nx']}x{inp['nz']} K={inp['K']}")
    d = observed_data(inp, torch, KKTProblem)
    p = KKTProblem.from_inputs(inp, reg_on_update=True)
    if not args.no_autotune:
        # shape of the block solver for this grid (setup, outside the timed region)
        table = p.autotune(prec="c64" if args.pc == "inexact" else "c128", solves_per_factor=100.0)
        log(args, "autotune: " + ", ".join(f"P={r['chunks']} ns={r['sources_per_group']}: "
                                            f"{r['t_factor_ms']:.1f}+100x{r['t_solve_ms']:.3f} ms"
                                            for r in table[:4]))
    opts = dict(rtol=args.rtol, restart=args.restart, maxit=600, pc=args.pc, fwd_prec="c128",
                update_in_place=True, want_xi=False)
    families = ["kkt_apply", "blu_factor", "blu_fwd_c64", "blu_bwd_c64", "blu_correct", "blu_chain",
                "blu_fwd_c128", "blu_bwd_c128"]
    # (blu_chain is a family of launches of unequal work: the reduction's levels)
    single = ["kkt_apply", "blu_fwd_c64", "blu_bwd_c64", "blu_correct", "blu_fwd_c128", "blu_bwd_c128"]
    # The last warm-up step records every kernel family (HIP events around each launch):
    # it gives the per-family breakdown and picks the single-kernel family with the largest
    # total time.  The timed steps then record that family only, so the other families'
    # events (thousands per step) do not weigh on the timed region.
    warm = None
    for w in range(args.warmup):
        last = w == args.warmup - 1
        if last:
            p.profile_enable(True)
        _, _, st = p.newton_step(d, **opts)
        if last:
            warm = {f: p.profile_read(f) for f in families}
            p.profile_enable(False)
        log(args, f"warmup {w}: iters={st['outer_iters']} rel={st['rel_res']:.2e} {st['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()
    if warm is not None:
        dominant = max((f for f in single if warm[f][0] > 0), key=lambda f: warm[f][1])
    else:   # no warm-up step: the family that dominates this workload in profiled runs
        dominant = "blu_correct" if args.pc == "inexact" else "blu_fwd_c128"
    p.profile_enable(True)
    p.profile_only(dominant)
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, _, st = p.newton_step(d, **opts)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom = p.profile_read(dominant)
    p.profile_only(None)
    p.profile_enable(False)
    for k, st in enumerate(stats):
        log(args, f"step {k}: iters={st['outer_iters']} (reorth {st['reorth_passes']}) rel={st['rel_res']:.2e} "
                  f"total={st['t_total_ms']:.1f} ms "
                  f"factor={st['t_factor_ms']:.1f} fwd={st['t_forward_ms']:.1f} pc={st['t_precond_ms']:.1f} "
                  f"mv={st['t_matvec_ms']:.1f} orth={st['t_orth_ms']:.1f} misfit={st['misfit_before']:.4f}")
    ms_per_step = elapsed / args.steps * 1e3
    roof = roofline_for(dominant, p, *dom)
    roof["traffic"] = measured_traffic(dominant, args.config)
    roof["events"] = "HIP events around this family's launches only, over the timed steps"
    kkt_here = roofline_for("kkt_apply", p, *warm["kkt_apply"]) if warm and warm["kkt_apply"][0] else None
    per_kernel = ({f: {"launches": n, "total_ms": ms, "avg_us": (ms / n * 1e3 if n else None)}
                   for f, (n, ms) in warm.items()} if warm else None)
    mean = lambda key: float(np.mean([s[key] for s in stats]))
    result = {
        "metric": "Newton-step time to KKT rel. res 1e-6",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 outer (FP64) + c64 block sweeps" if args.pc == "inexact" else "c128",
        "data": "synthetic",
        "config": {"workload": (f"{args.config}: {inp['nx']}x{inp['nz']} grid, h={inp['h']:g} m, "
                                f"{inp['npml']}-cell PML, faulted-lens model, {inp['K']} sources, "
                                f"{len(inp['rec_ix'])} receivers, {inp['freq']:g} Hz, "
                                f"{'inexact' if args.pc == 'inexact' else 'exact'} block-triangular "
                                f"preconditioner, FGMRES({args.restart}) to {args.rtol:g}, b_s = 0"),
                   "global_batch": inp["K"], "parallelism": "single GPU",
                   "solver_shape": dict(zip(("chunks", "sources_per_group"), p.solver_shape))},
        "roofline": roof,
        "breakdown_ms": {"factor": mean("t_factor_ms"), "forward": mean("t_forward_ms"),
                         "precond": mean("t_precond_ms"), "matvec": mean("t_matvec_ms"),
                         "orth": mean("t_orth_ms"), "outer_iters": mean("outer_iters"),
                         "rel_res": max(s["rel_res"] for s in stats),
                         "misfit_first": stats[0]["misfit_before"], "misfit_last": stats[-1]["misfit_before"]},
        "per_kernel_warmup_step": per_kernel,
        "kkt_apply": {"this_workload": kkt_here and {"GB_s": kkt_here["achieved"], "frac": kkt_here["frac"],
                                                      "note": "183 MB per call: Infinity-Cache resident"}},
    }
    if not args.no_hbm_kkt:
        p.close()
        result["kkt_apply"]["hbm"] = hbm_kkt(torch, KKTProblem, args)
    if not args.no_cpu_baseline:
        log(args, "timing the oracle on the host ...")
        result["cpu_baseline"] = cpu_baseline(inp, result["breakdown_ms"]["outer_iters"], args)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
