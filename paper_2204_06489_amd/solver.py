"""Python binding of the C ABI: argument marshalling on torch tensors only.

Every computation happens in libkktfwi.so (HIP kernels on gfx950).  Tensors must
live on the GPU, be contiguous and have the documented dtype; outputs are
allocated with torch and handed to the library as device pointers.  Work is
ordered on the current torch stream at construction time (see ``set_stream``).
"""

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (KF_C128, KF_C64, KF_MIXED, KF_PC_EXACT, KF_PC_INEXACT, KF_PC_MULTIGRID, KF_ENOCONV, KfCgOpts,
                   KfCgStats, KfDesc, KfMgStats, KfNewtonOpts, KfNewtonStats, KfSolveStats, check, lib)

_PREC = {"c128": KF_C128, "c64": KF_C64, "mixed": KF_MIXED}
_PC = {"exact": KF_PC_EXACT, "inexact": KF_PC_INEXACT, "multigrid": KF_PC_MULTIGRID}
_OUTER = {"fgmres": 0, "bicgstab": 1}


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class KKTProblem:
    """One frequency on one grid: A(gamma, omega) with PML, acquisition, weights and eps.

    Arguments follow ``kf_desc`` of the C ABI.  ``gamma`` is the full-grid squared
    slowness [nz][nx] (numpy or torch float64)."""

    def __init__(self, nx, nz, h, npml, omega, gamma, src_ix, src_iz, rec_ix, rec_iz, w=None, eps=1.0,
                 reg_on_update=True, pml_r0=1e-3, pml_cref=4000.0, stream=None):
        L = lib()
        self.nx, self.nz, self.npml, self.h, self.omega = int(nx), int(nz), int(npml), float(h), float(omega)
        self._src_ix = np.ascontiguousarray(src_ix, dtype=np.int32)
        self._src_iz = np.ascontiguousarray(src_iz, dtype=np.int32)
        self._rec_ix = np.ascontiguousarray(rec_ix, dtype=np.int32)
        self._rec_iz = np.ascontiguousarray(rec_iz, dtype=np.int32)
        self.K, self.nrec = len(self._src_ix), len(self._rec_ix)
        if len(self._src_iz) != self.K or len(self._rec_iz) != self.nrec:
            raise ValueError("source / receiver index arrays differ in length")
        self._w = None if w is None else np.ascontiguousarray(w, dtype=np.float64).reshape(self.K, self.nrec)
        d = KfDesc()
        d.nx, d.nz, d.h, d.npml = self.nx, self.nz, self.h, self.npml
        d.pml_r0, d.pml_cref, d.omega = float(pml_r0), float(pml_cref), self.omega
        d.K = self.K
        d.src_ix = self._src_ix.ctypes.data_as(C.POINTER(C.c_int32))
        d.src_iz = self._src_iz.ctypes.data_as(C.POINTER(C.c_int32))
        d.nrec = self.nrec
        d.rec_ix = self._rec_ix.ctypes.data_as(C.POINTER(C.c_int32))
        d.rec_iz = self._rec_iz.ctypes.data_as(C.POINTER(C.c_int32))
        d.w = self._w.ctypes.data_as(C.POINTER(C.c_double)) if self._w is not None else None
        d.eps = float(eps)
        d.reg_on_update = int(bool(reg_on_update))
        self.eps, self.reg_on_update = float(eps), bool(reg_on_update)
        self._h = C.c_void_p()
        if isinstance(gamma, torch.Tensor) and gamma.is_cuda:
            g = gamma.to(torch.float64).contiguous()
            check(L.kf_create(C.byref(d), C.c_void_p(g.data_ptr()), 1, _stream_handle(stream), C.byref(self._h)))
        else:
            g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
            if g.shape != (self.nz, self.nx):
                raise ValueError(f"gamma must be [{self.nz}][{self.nx}]")
            check(L.kf_create(C.byref(d), C.c_void_p(g.ctypes.data), 0, _stream_handle(stream), C.byref(self._h)))
        sz = (C.c_int64 * 6)()
        check(L.kf_sizes(self._h, sz))
        self.Ng, self.Nxi = int(sz[4]), int(sz[5])
        self.Nu = self.nx * self.nz
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_inputs(cls, inp, gamma=None, eps=None, K=None, reg_on_update=True, stream=None):
        """Build from a ``synthetic.make_problem_inputs`` dictionary."""
        K = inp["K"] if K is None else K
        return cls(inp["nx"], inp["nz"], inp["h"], inp["npml"], inp["omega"],
                   inp["gamma0"] if gamma is None else gamma, inp["src_ix"][:K], inp["src_iz"][:K],
                   inp["rec_ix"], inp["rec_iz"], w=np.asarray(inp["w"])[:K],
                   eps=inp["eps"] if eps is None else eps, reg_on_update=reg_on_update,
                   pml_r0=inp["pml_r0"], pml_cref=inp["pml_cref"], stream=stream)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- shapes -----------------------------------------------------------------
    @property
    def field_shape(self):
        return (self.K, self.nz, self.nx)

    def empty_field(self, dtype=torch.complex128):
        return torch.empty(self.field_shape, dtype=dtype, device=self.device)

    def empty_xi(self):
        return torch.empty(self.Nxi, dtype=torch.complex128, device=self.device)

    def pack(self, du, ds, lam):
        return torch.cat([du.reshape(-1), ds.reshape(-1), lam.reshape(-1)]).contiguous()

    def unpack(self, xi):
        n = self.K * self.Nu
        return (xi[:n].view(self.field_shape), xi[n:n + self.Ng], xi[n + self.Ng:].view(self.field_shape))

    # ---- state ------------------------------------------------------------------
    def set_stream(self, stream=None):
        check(lib().kf_set_stream(self._h, _stream_handle(stream)))

    def set_gamma(self, gamma):
        g = gamma.to(device=self.device, dtype=torch.float64).contiguous()
        check(lib().kf_set_gamma(self._h, _ptr(g, numel=self.Nu, name="gamma")))
        torch.cuda.current_stream().synchronize()
        self.gamma_token = getattr(self, "gamma_token", 0) + 1

    def get_gamma(self):
        out = torch.empty((self.nz, self.nx), dtype=torch.float64, device=self.device)
        check(lib().kf_get_gamma(self._h, _ptr(out)))
        return out

    def set_background(self, u):
        check(lib().kf_set_background(self._h, _ptr(u, torch.complex128, self.K * self.Nu, "u_n")))

    def get_background(self):
        out = self.empty_field()
        check(lib().kf_get_background(self._h, _ptr(out)))
        return out

    def factor(self, which=1):
        t = C.c_double()
        check(lib().kf_factor(self._h, int(which), C.byref(t)))
        return t.value

    def set_solver_shape(self, chunks=0, sources_per_group=0):
        """Column chunks of the partitioned block factorisation (0 = automatic) and
        right-hand sides per workgroup in the block solves (0 = 1)."""
        torch.cuda.current_stream().synchronize()
        check(lib().kf_set_solver_shape(self._h, int(chunks), int(sources_per_group)))

    def autotune(self, prec="c64", solves_per_factor=100.0):
        """Time solver shapes on this problem and keep the best (see kf_autotune).
        Returns the measured table as a list of dicts, best first."""
        from ._lib import KfTuneEntry
        torch.cuda.current_stream().synchronize()
        tab = (KfTuneEntry * 64)()
        n = C.c_int32()
        check(lib().kf_autotune(self._h, _PREC[prec], float(solves_per_factor), tab, 64, C.byref(n)))
        rows = [dict(chunks=e.chunks, sources_per_group=e.sources_per_group, t_factor_ms=e.t_factor_ms,
                     t_solve_ms=e.t_solve_ms, score_ms=e.score_ms) for e in tab[:min(n.value, 64)]]
        return sorted(rows, key=lambda r: r["score_ms"])

    @property
    def solver_shape(self):
        c, s = C.c_int32(), C.c_int32()
        check(lib().kf_get_solver_shape(self._h, C.byref(c), C.byref(s)))
        return c.value, s.value

    def sources(self):
        f = self.empty_field()
        check(lib().kf_sources(self._h, _ptr(f)))
        return f

    # ---- H-block of the preconditioner's middle stage ------------------------------
    def set_hblock(self, kind="eps", max_pairs=4):
        """"eps" (L = eps I) or "lbfgs" (L-BFGS from (ds, H ds) pairs of previous steps)."""
        check(lib().kf_set_hblock(self._h, {"eps": 0, "lbfgs": 1}[kind], int(max_pairs)))

    def hblock_add_pair(self, s, y):
        check(lib().kf_hblock_add_pair(self._h, _ptr(s, torch.complex128, self.Ng, "s"),
                                       _ptr(y, torch.complex128, self.Ng, "y")))

    # ---- shifted-Laplacian multigrid -----------------------------------------------
    def set_multigrid(self, prec="c64", beta=0.5, inner_rtol=1e-3, inner_maxit=200, n_min=20):
        check(lib().kf_set_multigrid(self._h, _PREC[prec], float(beta), float(inner_rtol), int(inner_maxit),
                                     int(n_min)))

    def helmholtz_solve_mg(self, rhs, adjoint=False, rtol=1e-3, maxit=200, out=None):
        """x with A x = rhs (A^H x = rhs) by multigrid-preconditioned BiCGStab; (x, stats)."""
        x = torch.empty_like(rhs) if out is None else out
        st = KfMgStats()
        s = check(lib().helmholtz_solve_mg(self._h, int(adjoint), _ptr(rhs, torch.complex128, self.K * self.Nu, "rhs"),
                                           _ptr(x, torch.complex128, self.K * self.Nu, "x"), float(rtol), int(maxit),
                                           C.byref(st)), allow=(KF_ENOCONV,))
        return x, {"iters": st.iters, "vcycles": st.vcycles, "levels": st.levels, "rel_res_max": st.rel_res_max,
                   "converged": s != KF_ENOCONV}

    def mg_vcycle(self, b):
        x = torch.empty_like(b)
        check(lib().kf_mg_vcycle(self._h, _ptr(b, torch.complex128, self.K * self.Nu, "b"), _ptr(x)))
        return x

    def mg_levels(self):
        dims = (C.c_int32 * 16)()
        n = C.c_int32()
        check(lib().kf_mg_levels(self._h, dims, C.byref(n)))
        return [(dims[2 * l], dims[2 * l + 1]) for l in range(n.value)]

    # ---- operators --------------------------------------------------------------
    def stencil_apply(self, x, adjoint=False):
        prec = KF_C128 if x.dtype == torch.complex128 else KF_C64
        y = torch.empty_like(x)
        check(lib().kf_stencil_apply(self._h, int(adjoint), prec, _ptr(x, numel=self.K * self.Nu, name="x"), _ptr(y)))
        return y

    def helmholtz_solve(self, rhs, adjoint=False, prec="c128", rtol=0.0, maxit=10, out=None):
        """x with A x = rhs (or A^H x = rhs) for all sources; returns (x, stats dict)."""
        pv = _PREC[prec]
        dt = torch.complex64 if pv == KF_C64 else torch.complex128
        x = torch.empty_like(rhs) if out is None else out
        st = KfSolveStats()
        s = check(lib().helmholtz_solve(self._h, int(adjoint), pv, _ptr(rhs, dt, self.K * self.Nu, "rhs"),
                                        _ptr(x, dt, self.K * self.Nu, "x"), float(rtol), int(maxit),
                                        C.byref(st)), allow=(KF_ENOCONV,))
        return x, {"iters": st.iters, "rel_res_max": st.rel_res_max, "converged": s != KF_ENOCONV}

    def kkt_apply(self, xi, out=None):
        y = self.empty_xi() if out is None else out
        check(lib().kkt_apply(self._h, _ptr(xi, torch.complex128, self.Nxi, "xi"), _ptr(y, numel=self.Nxi)))
        return y

    def precond_apply(self, y, pc="exact", out=None):
        z = self.empty_xi() if out is None else out
        check(lib().precond_apply(self._h, _PC[pc], _ptr(y, torch.complex128, self.Nxi, "y"),
                                  _ptr(z, numel=self.Nxi)))
        return z

    def newton_step(self, d_obs, rtol=1e-6, restart=30, maxit=200, pc="exact", fwd_prec="c128",
                    fwd_rtol=1e-10, misfit_after=False, update_in_place=True, want_xi=True, reorth_eta=0.1,
                    outer="fgmres"):
        """One full-space GN step; returns (xi or None, gamma_{n+1}, stats dict).
        reorth_eta: second Gram-Schmidt pass when |w'| < reorth_eta |w| (1 = always).
        outer: "fgmres" or "bicgstab" (the KKT solver)."""
        o = KfNewtonOpts()
        o.rtol, o.restart, o.maxit, o.pc = float(rtol), int(restart), int(maxit), _PC[pc]
        o.fwd_prec, o.fwd_rtol, o.misfit_after = _PREC[fwd_prec], float(fwd_rtol), int(bool(misfit_after))
        o.reorth_eta = float(reorth_eta)
        o.outer = _OUTER[outer]
        xi = self.empty_xi() if want_xi else None
        g1 = torch.empty((self.nz, self.nx), dtype=torch.float64, device=self.device)
        st = KfNewtonStats()
        s = check(lib().newton_step(self._h, _ptr(d_obs, torch.complex128, self.K * self.nrec, "d_obs"),
                                    C.byref(o), _ptr(xi) if xi is not None else None, _ptr(g1),
                                    int(bool(update_in_place)), C.byref(st)), allow=(KF_ENOCONV,))
        if update_in_place:
            self.gamma_token = getattr(self, "gamma_token", 0) + 1
        stats = {f: getattr(st, f) for f, _ in KfNewtonStats._fields_ if f != "rel_res_hist"}
        stats["rel_res_hist"] = list(st.rel_res_hist[:max(0, st.outer_iters)])
        stats["converged"] = s != KF_ENOCONV
        return xi, g1, stats

    def rsgn_step(self, d_obs, rtol=1e-6, maxit=500, solve_prec="c128", solve_rtol=1e-10, real_constrained=False,
                  fwd_prec="c128", fwd_rtol=1e-10, update_in_place=True, want_ds=True):
        """Reduced-space GN step by CG on the normal equations (rsgn_cg_step); returns
        (ds or None, gamma_{n+1}, stats dict)."""
        o = KfCgOpts()
        o.rtol, o.maxit, o.solve_prec, o.solve_rtol = float(rtol), int(maxit), _PREC[solve_prec], float(solve_rtol)
        o.real_constrained, o.fwd_prec, o.fwd_rtol = int(bool(real_constrained)), _PREC[fwd_prec], float(fwd_rtol)
        ds = torch.empty(self.Ng, dtype=torch.complex128, device=self.device) if want_ds else None
        g1 = torch.empty((self.nz, self.nx), dtype=torch.float64, device=self.device)
        st = KfCgStats()
        s = check(lib().rsgn_cg_step(self._h, _ptr(d_obs, torch.complex128, self.K * self.nrec, "d_obs"),
                                     C.byref(o), _ptr(ds) if ds is not None else None, _ptr(g1),
                                     int(bool(update_in_place)), C.byref(st)), allow=(KF_ENOCONV,))
        if update_in_place:
            self.gamma_token = getattr(self, "gamma_token", 0) + 1
        stats = {f: getattr(st, f) for f, _ in KfCgStats._fields_ if f != "rel_res_hist"}
        stats["rel_res_hist"] = list(st.rel_res_hist[:max(0, min(st.iters, 512))])
        stats["converged"] = s != KF_ENOCONV
        return ds, g1, stats

    def adjoint_gradient(self, u, grad_u, prec="c128"):
        pv = _PREC[prec]
        dt = torch.complex64 if pv == KF_C64 else torch.complex128
        g = torch.empty((self.nz, self.nx), dtype=torch.float64, device=self.device)
        check(lib().helmholtz_adjoint_gradient(self._h, pv, _ptr(u, dt, self.K * self.Nu, "u"),
                                               _ptr(grad_u, dt, self.K * self.Nu, "grad_u"), _ptr(g)))
        return g

    # ---- profiling --------------------------------------------------------------
    def profile_enable(self, on=True):
        check(lib().kf_profile_enable(self._h, int(bool(on))))

    def profile_read(self, name):
        n, ms = C.c_int64(), C.c_double()
        check(lib().kf_profile_read(self._h, name.encode(), C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    def profile_work(self, name):
        """Algorithmic work (bytes) the library counted for a kernel family's recorded launches."""
        w = C.c_double()
        check(lib().kf_profile_work(self._h, name.encode(), C.byref(w)))
        return float(w.value)

    def profile_only(self, name=None):
        """Record one kernel family only (None: all families)."""
        check(lib().kf_profile_only(self._h, (name or "").encode()))


def newton_step_concurrent(problems, d_obs, rtol=1e-6, restart=30, maxit=200, pc="exact", fwd_prec="c128",
                           fwd_rtol=1e-10, misfit_after=False, update_in_place=True, want_xi=True, reorth_eta=0.1,
                           outer="fgmres"):
    """One Newton step on each of several independent problems at once
    (newton_step_concurrent: a stream and a host thread per problem).  Returns
    (list of xi or None, list of gamma_{n+1}, list of stats dicts, each with "converged")."""
    n = len(problems)
    o = KfNewtonOpts()
    o.rtol, o.restart, o.maxit, o.pc = float(rtol), int(restart), int(maxit), _PC[pc]
    o.fwd_prec, o.fwd_rtol, o.misfit_after = _PREC[fwd_prec], float(fwd_rtol), int(bool(misfit_after))
    o.reorth_eta = float(reorth_eta)
    o.outer = _OUTER[outer]
    xis = [q.empty_xi() if want_xi else None for q in problems]
    gs = [torch.empty((q.nz, q.nx), dtype=torch.float64, device=q.device) for q in problems]
    arr = (C.c_void_p * n)(*[q._h.value for q in problems])
    dp = (C.c_void_p * n)(*[_ptr(d, torch.complex128, q.K * q.nrec, "d_obs").value for d, q in zip(d_obs, problems)])
    xp = (C.c_void_p * n)(*[_ptr(x).value if x is not None else None for x in xis])
    gp = (C.c_void_p * n)(*[_ptr(g).value for g in gs])
    st = (KfNewtonStats * n)()
    torch.cuda.current_stream().synchronize()   # the outputs' allocation is complete
    s = check(lib().newton_step_concurrent(arr, n, dp, C.byref(o), xp, gp, int(bool(update_in_place)), st),
              allow=(KF_ENOCONV,))
    stats = []
    for k in range(n):
        d = {f: getattr(st[k], f) for f, _ in KfNewtonStats._fields_ if f != "rel_res_hist"}
        d["rel_res_hist"] = list(st[k].rel_res_hist[:max(0, st[k].outer_iters)])
        d["converged"] = s != KF_ENOCONV or st[k].rel_res <= rtol
        stats.append(d)
    if update_in_place:
        for q in problems:
            q.gamma_token = getattr(q, "gamma_token", 0) + 1
    return xis, gs, stats


def newton_continuation(problems, d_obs, steps, rtol=1e-6, restart=30, maxit=200, pc="exact", fwd_prec="c128",
                        fwd_rtol=1e-10, reorth_eta=0.1):
    """Frequency continuation (newton_continuation): steps[q] Newton steps on problems[q],
    each problem starting from the model the previous one reached.  Returns (final gamma,
    list of per-step stats dicts)."""
    n = len(problems)
    o = KfNewtonOpts()
    o.rtol, o.restart, o.maxit, o.pc = float(rtol), int(restart), int(maxit), _PC[pc]
    o.fwd_prec, o.fwd_rtol, o.misfit_after = _PREC[fwd_prec], float(fwd_rtol), 0
    o.reorth_eta = float(reorth_eta)
    last = problems[-1]
    g = torch.empty((last.nz, last.nx), dtype=torch.float64, device=last.device)
    arr = (C.c_void_p * n)(*[q._h.value for q in problems])
    dp = (C.c_void_p * n)(*[_ptr(d, torch.complex128, q.K * q.nrec, "d_obs").value for d, q in zip(d_obs, problems)])
    sp = (C.c_int32 * n)(*[int(s) for s in steps])
    total = sum(int(s) for s in steps)
    st = (KfNewtonStats * max(total, 1))()
    torch.cuda.current_stream().synchronize()
    check(lib().newton_continuation(arr, n, dp, sp, C.byref(o), _ptr(g), st))
    out = []
    for k in range(total):
        d = {f: getattr(st[k], f) for f, _ in KfNewtonStats._fields_ if f != "rel_res_hist"}
        d["rel_res_hist"] = list(st[k].rel_res_hist[:max(0, st[k].outer_iters)])
        out.append(d)
    for q in problems:
        q.gamma_token = getattr(q, "gamma_token", 0) + 1
    return g, out


class KKTBatch:
    """Several problems (e.g. one per frequency, on uneven grids) advanced together.

    Factorisations and block solves of all problems are single persistent launches;
    ``newton_step`` runs the problems' FGMRES iterations in lockstep, optionally
    replaying each Krylov column's preconditioner and KKT matvec from a captured
    hipGraph.  The batch orders all work on one stream (the problems' streams are
    set to it, and given back when the batch is closed); destroy the batch before its
    problems.  While the batch exists, a member's own calls run on the batch's stream:
    close the batch (or synchronize) before reading their results on another stream."""

    def __init__(self, problems, stream=None):
        self.problems = list(problems)
        n = len(self.problems)
        arr = (C.c_void_p * n)(*[q._h.value for q in self.problems])
        self._b = C.c_void_p()
        # a stream of the batch's own (None): the library creates a capturable one
        h = C.c_void_p(stream.cuda_stream) if stream is not None else C.c_void_p(None)
        check(lib().kf_batch_create(arr, n, h, C.byref(self._b)))

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().kf_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self, which=1):
        t = C.c_double()
        torch.cuda.current_stream().synchronize()
        check(lib().kf_batch_factor(self._b, int(which), C.byref(t)))
        return t.value

    def helmholtz_solve(self, rhs, adjoint=False, prec="c128"):
        pv = _PREC[prec]
        dt = torch.complex64 if pv == KF_C64 else torch.complex128
        xs = [torch.empty_like(r) for r in rhs]
        n = len(self.problems)
        torch.cuda.current_stream().synchronize()   # inputs from the caller's stream are complete
        rp = (C.c_void_p * n)(*[_ptr(r, dt, q.K * q.Nu, "rhs").value for r, q in zip(rhs, self.problems)])
        xp = (C.c_void_p * n)(*[_ptr(x).value for x in xs])
        check(lib().helmholtz_solve_batched(self._b, int(adjoint), pv, rp, xp))
        return xs

    def newton_step(self, d_obs, rtol=1e-6, restart=30, maxit=200, pc="exact", update_in_place=True,
                    use_graph=True, want_xi=True, reorth_eta=0.1):
        """Returns (list of xi or None, list of gamma_{n+1}, list of stats dicts)."""
        n = len(self.problems)
        o = KfNewtonOpts()
        o.rtol, o.restart, o.maxit, o.pc = float(rtol), int(restart), int(maxit), _PC[pc]
        o.fwd_prec, o.fwd_rtol, o.misfit_after = KF_C128, 1e-10, 0
        o.reorth_eta = float(reorth_eta)
        xis = [q.empty_xi() for q in self.problems] if want_xi else [None] * n
        gs = [torch.empty((q.nz, q.nx), dtype=torch.float64, device=q.device) for q in self.problems]
        dp = (C.c_void_p * n)(*[_ptr(d, torch.complex128, q.K * q.nrec, "d_obs").value
                                for d, q in zip(d_obs, self.problems)])
        xp = (C.c_void_p * n)(*[(x.data_ptr() if x is not None else None) for x in xis])
        gp = (C.c_void_p * n)(*[g.data_ptr() for g in gs])
        st = (KfNewtonStats * n)()
        torch.cuda.current_stream().synchronize()   # inputs from the caller's stream are complete
        s = check(lib().newton_step_batched(self._b, dp, C.byref(o), xp, gp, int(bool(update_in_place)),
                                            int(bool(use_graph)), st), allow=(KF_ENOCONV,))
        out = []
        for k in range(n):
            d = {f: getattr(st[k], f) for f, _ in KfNewtonStats._fields_ if f != "rel_res_hist"}
            d["rel_res_hist"] = list(st[k].rel_res_hist[:max(0, st[k].outer_iters)])
            d["converged"] = s != KF_ENOCONV
            out.append(d)
        if update_in_place:
            for q in self.problems:
                q.gamma_token = getattr(q, "gamma_token", 0) + 1
        return xis, gs, out
