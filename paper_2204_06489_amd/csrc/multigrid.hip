// Shifted-Laplacian multigrid: the inexact block solver A~ of the third preconditioner
// variant (Section 5 names the shifted-Laplacian preconditioner, inverted approximately
// by multigrid, as the better A~ for eq. precond_approx).
//
// Every source's solve A x_k = b_k runs BiCGStab (van der Vorst) right-preconditioned by
// one V-cycle of the shifted operator M = A(gamma (1 + i beta)); all K sources advance in
// lock step, each with its own scalars, and a converged source stops moving.  The
// hierarchy: standard coarsening of the vertex grid (n -> (n + 1) / 2 while both sizes
// are odd and the smaller is at least n_min), spacing doubled, PML width halved, gamma
// injected; every level's operator is the shifted 5-point PML stencil rediscretised on its
// grid (coefficients on the fly from 1-D stretch arrays and gamma, like A itself).
// Smoothing: a z-line Jacobi sweep (one thread per grid column and source solves its
// tridiagonal line by the Thomas algorithm, the x-neighbours from the previous iterate),
// then an x-line sweep (one thread per row); the reverse order after the coarse
// correction.  Full-weighting restriction, bilinear prolongation.  The coarsest level is a
// problem of its own, factorised by the partitioned block LU with the shift, and solved
// exactly.  A^H x = b is solved as A conj(x) = conj(b) (A is complex symmetric).
//
// R is the arithmetic of the multigrid and BiCGStab fields (float: complex64 with FP32
// arithmetic; double: complex128); per-source inner products accumulate in FP64.
#include "common.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace {

constexpr int TB = 256;

// ---------------------------------------------------------------------------
// level kernels ([K][nz][nx] fields, x fastest)
// ---------------------------------------------------------------------------
template <typename R>
__device__ inline void stencil_R(const Grid &g, int i, int j, cplx<R> &cc, cplx<R> &cxm, cplx<R> &cxp,
                                 cplx<R> &czm, cplx<R> &czp) {
  const Stencil5 s = stencil_at(g, i, j);
  cc = ccast<R>(s.cc); cxm = ccast<R>(s.cxm); cxp = ccast<R>(s.cxp); czm = ccast<R>(s.czm); czp = ccast<R>(s.czp);
}

// Smith's complex division in R
template <typename R> __device__ inline cplx<R> cdivR(cplx<R> a, cplx<R> b) {
  if (fabs(b.x) >= fabs(b.y)) {
    R r = b.y / b.x, d = b.x + b.y * r;
    return mk<R>((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  R r = b.x / b.y, d = b.x * r + b.y;
  return mk<R>((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// r = b - M x
template <typename R>
__global__ __launch_bounds__(TB) void k_mg_residual(Grid g, int K, const cplx<R> *__restrict__ x,
                                                    const cplx<R> *__restrict__ b, cplx<R> *__restrict__ r) {
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t t = (size_t)blockIdx.x * TB + threadIdx.x;
  if (t >= (size_t)K * Nu) return;
  const size_t p = t % Nu;
  const int j = (int)(p / g.nx), i = (int)(p - (size_t)j * g.nx);
  cplx<R> cc, cxm, cxp, czm, czp;
  stencil_R<R>(g, i, j, cc, cxm, cxp, czm, czp);
  cplx<R> acc = cmul(cc, x[t]);
  if (i > 0) cfma(acc, cxm, x[t - 1]);
  if (i + 1 < g.nx) cfma(acc, cxp, x[t + 1]);
  if (j > 0) cfma(acc, czm, x[t - g.nx]);
  if (j + 1 < g.nz) cfma(acc, czp, x[t + g.nx]);
  r[t] = csub(b[t], acc);
}

// One z-line Jacobi sweep: for every grid column i and source k (one thread each) solve
//   czm_j y_{j-1} + cc_j y_j + czp_j y_{j+1} = b_j - cxm_j x(i-1, j) - cxp_j x(i+1, j)
// by the Thomas algorithm; the forward sweep's ratios go to cp, its values to y.
// x == nullptr stands for x = 0.
template <typename R>
__global__ __launch_bounds__(TB) void k_mg_zline(Grid g, int K, const cplx<R> *__restrict__ x,
                                                 const cplx<R> *__restrict__ b, cplx<R> *__restrict__ y,
                                                 cplx<R> *__restrict__ cp) {
  const int t = blockIdx.x * TB + threadIdx.x;
  if (t >= K * g.nx) return;
  const int k = t / g.nx, i = t - k * g.nx;
  const size_t Nu = (size_t)g.nx * g.nz, base = (size_t)k * Nu + i;
  cplx<R> cprev = mk<R>(0, 0), dprev = mk<R>(0, 0);
  for (int j = 0; j < g.nz; ++j) {
    const size_t o = base + (size_t)j * g.nx;
    cplx<R> cc, cxm, cxp, czm, czp;
    stencil_R<R>(g, i, j, cc, cxm, cxp, czm, czp);
    cplx<R> rhs = b[o];
    if (x) {
      if (i > 0) rhs = csub(rhs, cmul(cxm, x[o - 1]));
      if (i + 1 < g.nx) rhs = csub(rhs, cmul(cxp, x[o + 1]));
    }
    if (j == 0) czm = mk<R>(0, 0);
    const cplx<R> den = csub(cc, cmul(czm, cprev));
    const cplx<R> c = j + 1 < g.nz ? cdivR<R>(czp, den) : mk<R>(0, 0);
    const cplx<R> d = cdivR<R>(csub(rhs, cmul(czm, dprev)), den);
    cp[o] = c;
    y[o] = d;
    cprev = c;
    dprev = d;
  }
  cplx<R> nxt = mk<R>(0, 0);
  for (int j = g.nz - 1; j >= 0; --j) {
    const size_t o = base + (size_t)j * g.nx;
    const cplx<R> v = csub(y[o], cmul(cp[o], nxt));
    y[o] = v;
    nxt = v;
  }
}

// One x-line Jacobi sweep: every grid row j and source k (one thread each), the
// z-neighbours from x.
template <typename R>
__global__ __launch_bounds__(TB) void k_mg_xline(Grid g, int K, const cplx<R> *__restrict__ x,
                                                 const cplx<R> *__restrict__ b, cplx<R> *__restrict__ y,
                                                 cplx<R> *__restrict__ cp) {
  const int t = blockIdx.x * TB + threadIdx.x;
  if (t >= K * g.nz) return;
  const int k = t / g.nz, j = t - k * g.nz;
  const size_t Nu = (size_t)g.nx * g.nz, base = (size_t)k * Nu + (size_t)j * g.nx;
  cplx<R> cprev = mk<R>(0, 0), dprev = mk<R>(0, 0);
  for (int i = 0; i < g.nx; ++i) {
    const size_t o = base + i;
    cplx<R> cc, cxm, cxp, czm, czp;
    stencil_R<R>(g, i, j, cc, cxm, cxp, czm, czp);
    cplx<R> rhs = b[o];
    if (j > 0) rhs = csub(rhs, cmul(czm, x[o - g.nx]));
    if (j + 1 < g.nz) rhs = csub(rhs, cmul(czp, x[o + g.nx]));
    if (i == 0) cxm = mk<R>(0, 0);
    const cplx<R> den = csub(cc, cmul(cxm, cprev));
    const cplx<R> c = i + 1 < g.nx ? cdivR<R>(cxp, den) : mk<R>(0, 0);
    const cplx<R> d = cdivR<R>(csub(rhs, cmul(cxm, dprev)), den);
    cp[o] = c;
    y[o] = d;
    cprev = c;
    dprev = d;
  }
  cplx<R> nxt = mk<R>(0, 0);
  for (int i = g.nx - 1; i >= 0; --i) {
    const size_t o = base + i;
    const cplx<R> v = csub(y[o], cmul(cp[o], nxt));
    y[o] = v;
    nxt = v;
  }
}

// The same x-line sweep with one workgroup per grid row and source: the row's
// tridiagonal system is held in LDS and solved by parallel cyclic reduction (every
// equation eliminates its neighbours at distance s = 1, 2, 4, ... in log2 nx steps), so
// K nz workgroups share the chip instead of K nz threads.  Rows of up to PCR_MAX nodes.
constexpr int PCR_T = 256, PCR_E = 4, PCR_MAX = PCR_T * PCR_E;
template <typename R>
__global__ __launch_bounds__(PCR_T) void k_mg_xline_pcr(Grid g, int K, const cplx<R> *__restrict__ x,
                                                        const cplx<R> *__restrict__ b, cplx<R> *__restrict__ y) {
  using C = cplx<R>;
  extern __shared__ unsigned char smem_pcr[];
  const int nx = g.nx;
  C *A = (C *)smem_pcr, *B = A + nx, *Cu = B + nx, *D = Cu + nx;
  const int line = blockIdx.x;
  if (line >= K * g.nz) return;   // uniform
  const int k = line / g.nz, j = line - k * g.nz;
  const size_t Nu = (size_t)nx * g.nz, base = (size_t)k * Nu + (size_t)j * nx;
  const int tid = threadIdx.x;
  for (int i = tid; i < nx; i += PCR_T) {
    C cc, cxm, cxp, czm, czp;
    stencil_R<R>(g, i, j, cc, cxm, cxp, czm, czp);
    const size_t o = base + i;
    C rhs = b[o];
    if (j > 0) rhs = csub(rhs, cmul(czm, x[o - nx]));
    if (j + 1 < g.nz) rhs = csub(rhs, cmul(czp, x[o + nx]));
    A[i] = i > 0 ? cxm : mk<R>(0, 0);
    B[i] = cc;
    Cu[i] = i + 1 < nx ? cxp : mk<R>(0, 0);
    D[i] = rhs;
  }
  __syncthreads();
  for (int s = 1; s < nx; s <<= 1) {
    C na[PCR_E], nb[PCR_E], nc[PCR_E], nd[PCR_E];
#pragma unroll
    for (int u = 0; u < PCR_E; ++u) {
      const int i = tid + u * PCR_T;
      if (i < nx) {
        C bi = B[i], di = D[i], an = mk<R>(0, 0), cn = mk<R>(0, 0);
        if (i - s >= 0) {
          const C al = csub(mk<R>(0, 0), cdivR<R>(A[i], B[i - s]));
          an = cmul(al, A[i - s]);
          bi = cadd(bi, cmul(al, Cu[i - s]));
          di = cadd(di, cmul(al, D[i - s]));
        }
        if (i + s < nx) {
          const C ga = csub(mk<R>(0, 0), cdivR<R>(Cu[i], B[i + s]));
          cn = cmul(ga, Cu[i + s]);
          bi = cadd(bi, cmul(ga, A[i + s]));
          di = cadd(di, cmul(ga, D[i + s]));
        }
        na[u] = an; nb[u] = bi; nc[u] = cn; nd[u] = di;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PCR_E; ++u) {
      const int i = tid + u * PCR_T;
      if (i < nx) { A[i] = na[u]; B[i] = nb[u]; Cu[i] = nc[u]; D[i] = nd[u]; }
    }
    __syncthreads();
  }
  for (int i = tid; i < nx; i += PCR_T) y[base + i] = cdivR<R>(D[i], B[i]);
}

// full weighting: bc(I, J) = sum_{a, b in -1..1} w_a w_b r(2I + a, 2J + b) / 4, w = (1/2, 1, 1/2)
template <typename R>
__global__ __launch_bounds__(TB) void k_mg_restrict(int K, int nx, int nz, int ncx, int ncz,
                                                    const cplx<R> *__restrict__ r, cplx<R> *__restrict__ bc) {
  const size_t Nc = (size_t)ncx * ncz;
  const size_t t = (size_t)blockIdx.x * TB + threadIdx.x;
  if (t >= (size_t)K * Nc) return;
  const int k = (int)(t / Nc);
  const size_t q = t - (size_t)k * Nc;
  const int J = (int)(q / ncx), I = (int)(q - (size_t)J * ncx);
  const cplx<R> *rk = r + (size_t)k * nx * nz;
  cplx<R> acc = mk<R>(0, 0);
  for (int b = -1; b <= 1; ++b) {
    const int j = 2 * J + b;
    if (j < 0 || j >= nz) continue;
    const R wb = b == 0 ? R(1) : R(0.5);
    for (int a = -1; a <= 1; ++a) {
      const int i = 2 * I + a;
      if (i < 0 || i >= nx) continue;
      const R w = wb * (a == 0 ? R(1) : R(0.5)) * R(0.25);
      const cplx<R> v = rk[(size_t)j * nx + i];
      acc.x += w * v.x;
      acc.y += w * v.y;
    }
  }
  bc[t] = acc;
}

// bilinear prolongation added to the fine field: x(i, j) += sum of the coarse values of the
// cell corners around (i, j) with weights 1, 1/2 or 1/4
template <typename R>
__global__ __launch_bounds__(TB) void k_mg_prolong_add(int K, int nx, int nz, int ncx, int ncz,
                                                       const cplx<R> *__restrict__ ec, cplx<R> *__restrict__ x) {
  const size_t Nu = (size_t)nx * nz;
  const size_t t = (size_t)blockIdx.x * TB + threadIdx.x;
  if (t >= (size_t)K * Nu) return;
  const int k = (int)(t / Nu);
  const size_t p = t - (size_t)k * Nu;
  const int j = (int)(p / nx), i = (int)(p - (size_t)j * nx);
  const cplx<R> *e = ec + (size_t)k * ncx * ncz;
  const int I0 = i >> 1, J0 = j >> 1;
  const int I1 = (i & 1) ? I0 + 1 : I0, J1 = (j & 1) ? J0 + 1 : J0;
  const R wi = (i & 1) ? R(0.5) : R(1), wj = (j & 1) ? R(0.5) : R(1);
  cplx<R> v = mk<R>(0, 0);
  auto add = [&](int I, int J, R w) {
    if (I < ncx && J < ncz) {
      const cplx<R> c = e[(size_t)J * ncx + I];
      v.x += w * c.x;
      v.y += w * c.y;
    }
  };
  add(I0, J0, wi * wj);
  if (I1 != I0) add(I1, J0, wi * wj);
  if (J1 != J0) add(I0, J1, wi * wj);
  if (I1 != I0 && J1 != J0) add(I1, J1, wi * wj);
  x[t] = cadd(x[t], v);
}

// gamma of the next level: every second node
__global__ void k_mg_inject(int nx, int ncx, int ncz, const double *__restrict__ g, double *__restrict__ gc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncx * ncz) return;
  const int J = t / ncx, I = t - J * ncx;
  gc[t] = g[(size_t)(2 * J) * nx + 2 * I];
}

// c128 <-> R copies, conjugating for the adjoint
template <typename R>
__global__ void k_mg_in(int64_t n, int conj, const double2 *__restrict__ a, cplx<R> *__restrict__ b) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = mk<R>((R)a[t].x, (R)(conj ? -a[t].y : a[t].y));
}
template <typename R>
__global__ void k_mg_out(int64_t n, int conj, const cplx<R> *__restrict__ a, double2 *__restrict__ b) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = make_double2((double)a[t].x, conj ? -(double)a[t].y : (double)a[t].y);
}

// ---------------------------------------------------------------------------
// BiCGStab kernels: per-source inner products (FP64 accumulation, fixed order) and
// updates with per-source coefficients
// ---------------------------------------------------------------------------
constexpr int DB = 64;   // blocks per source of the inner products

// partial[k][blk][0..1] = sum conj(a) b over the block's share of source k
template <typename R>
__global__ __launch_bounds__(TB) void k_src_dot(size_t n_per, const cplx<R> *__restrict__ a,
                                                const cplx<R> *__restrict__ b, double *partial) {
  __shared__ double sr[TB], si[TB];
  const int k = blockIdx.y;
  const cplx<R> *ak = a + (size_t)k * n_per, *bk = b + (size_t)k * n_per;
  double re = 0.0, im = 0.0;
  for (size_t t = (size_t)blockIdx.x * TB + threadIdx.x; t < n_per; t += (size_t)DB * TB) {
    const double ax = ak[t].x, ay = ak[t].y, bx = bk[t].x, by = bk[t].y;
    re += ax * bx + ay * by;
    im += ax * by - ay * bx;
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((size_t)k * DB + blockIdx.x) * 2] = sr[0];
    partial[((size_t)k * DB + blockIdx.x) * 2 + 1] = si[0];
  }
}
__global__ void k_src_dot_finish(int K, const double *__restrict__ partial, double2 *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < DB; ++b) {
    re += partial[((size_t)k * DB + b) * 2];
    im += partial[((size_t)k * DB + b) * 2 + 1];
  }
  out[k] = make_double2(re, im);
}

// Per-source scalars of one BiCGStab iteration, in FP64:
//   stage 0 (before p):  rho_new = (rhat, r);  beta = (rho_new / rho) (alpha / omega)
//   stage 1 (after v):   alpha = rho_new / (rhat, v)
//   stage 2 (after t):   omega = (t, s) / (t, t);  rho = rho_new
// sc[k] = {rho, alpha, omega, rho_new, beta, active(1/0)} as complex values; a source
// whose denominator vanishes (breakdown, or an exact solution) stops (active = 0) and
// takes zero updates from then on.
__global__ void k_bicg_scalars(int K, int stage, const double2 *__restrict__ d0, const double2 *__restrict__ d1,
                               double2 *sc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 *s = sc + (size_t)k * 6;
  if (s[5].x == 0.0) {   // inactive: zero coefficients
    s[1] = s[2] = s[4] = make_double2(0.0, 0.0);
    return;
  }
  if (stage == 0) {
    const double2 rn = d0[k];
    s[3] = rn;
    if (cabs2(s[0]) == 0.0 || cabs2(s[2]) == 0.0) { s[5].x = 0.0; s[1] = s[2] = s[4] = make_double2(0, 0); return; }
    s[4] = cmul(cdiv(rn, s[0]), cdiv(s[1], s[2]));
  } else if (stage == 1) {
    const double2 den = d0[k];
    if (cabs2(den) == 0.0) { s[5].x = 0.0; s[1] = s[2] = s[4] = make_double2(0, 0); return; }
    s[1] = cdiv(s[3], den);
  } else {
    const double2 ts = d0[k], tt = d1[k];
    s[2] = tt.x > 0.0 ? cdiv(ts, tt) : make_double2(0.0, 0.0);
    s[0] = s[3];
  }
}

// p = r + beta (p - omega v)          (mode 0)
// s = r - alpha v                     (mode 1; s written to `out`)
// x += alpha ph + omega sh; r = s - omega t   (mode 2)
template <typename R>
__global__ __launch_bounds__(TB) void k_bicg_update(int mode, size_t n_per, int K, const double2 *__restrict__ sc,
                                                    cplx<R> *a, cplx<R> *b, cplx<R> *c, cplx<R> *d, cplx<R> *e,
                                                    cplx<R> *f) {
  const size_t t = (size_t)blockIdx.x * TB + threadIdx.x;
  if (t >= n_per * K) return;
  const int k = (int)(t / n_per);
  const double2 *s = sc + (size_t)k * 6;
  if (mode == 0) {   // a = p, b = r, c = v
    const cplx<R> beta = ccast<R>(s[4]), om = ccast<R>(s[2]);
    a[t] = cadd(b[t], cmul(beta, csub(a[t], cmul(om, c[t]))));
  } else if (mode == 1) {   // a = s(out), b = r, c = v
    const cplx<R> al = ccast<R>(s[1]);
    a[t] = csub(b[t], cmul(al, c[t]));
  } else {   // a = x, b = ph, c = sh, d = r, e = s, f = t
    const cplx<R> al = ccast<R>(s[1]), om = ccast<R>(s[2]);
    a[t] = cadd(a[t], cadd(cmul(al, b[t]), cmul(om, c[t])));
    d[t] = csub(e[t], cmul(om, f[t]));
  }
}

inline unsigned nblk(size_t n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace

#define CHECK_ST(expr)                  \
  do {                                  \
    kf_status s_ = (expr);              \
    if (s_ != KF_OK) return s_;         \
  } while (0)
#define LAUNCH_CHECK()                                                              \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) {                                                         \
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_));     \
      return KF_EHIP;                                                               \
    }                                                                               \
  } while (0)

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
struct MgLevel {
  int nx = 0, nz = 0, npml = 0;
  double h = 0.0;
  double *gamma = nullptr;                                  // owned except on level 0
  double2 *xn = nullptr, *ixh = nullptr, *zn = nullptr, *izh = nullptr;   // owned except on level 0
  void *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr, *cp = nullptr;   // R fields [K][nz][nx]
  Grid grid(double omega, double beta) const { return Grid{nx, nz, npml, h, omega, gamma, xn, ixh, zn, izh, beta}; }
};

struct MgState {
  int prec = KF_C64;            // KF_C64: complex64 fields, FP32 arithmetic; KF_C128: complex128
  double beta = 0.5, rtol = 1e-3;
  int maxit = 200, n_min = 20;
  std::vector<MgLevel> lev;
  kf_problem *coarse = nullptr; // the coarsest level, factorised with the shift
  uint64_t version = ~0ull;     // gamma version the hierarchy was built for
  void *bf[9] = {};             // BiCGStab fields: x, r, rhat, p, v, s, t, ph, sh
  double *partial = nullptr;    // inner-product partials [2][K][DB][2]
  double2 *dots = nullptr;      // [2][K]
  double2 *sc = nullptr;        // [K][6] per-source scalars
  double *host = nullptr;       // pinned [K] residual norms
};

static size_t fsz(const MgState *m) { return m->prec == KF_C64 ? sizeof(float2) : sizeof(double2); }

static void mg_free_fields(MgState *m) {
  for (size_t l = 0; l < m->lev.size(); ++l) {
    MgLevel &L = m->lev[l];
    for (void **q : {&L.b, &L.xa, &L.xb, &L.r, &L.cp})
      if (*q) { hipFree(*q); *q = nullptr; }
    if (l > 0) {
      for (void *q : {(void *)L.gamma, (void *)L.xn, (void *)L.ixh, (void *)L.zn, (void *)L.izh})
        if (q) hipFree(q);
      L.gamma = nullptr; L.xn = L.ixh = L.zn = L.izh = nullptr;
    }
  }
  m->lev.clear();
  for (void *&q : m->bf)
    if (q) { hipFree(q); q = nullptr; }
  if (m->partial) hipFree(m->partial);
  if (m->dots) hipFree(m->dots);
  if (m->sc) hipFree(m->sc);
  if (m->host) hipHostFree(m->host);
  m->partial = nullptr; m->dots = nullptr; m->sc = nullptr; m->host = nullptr;
  if (m->coarse) { kf_destroy(m->coarse); m->coarse = nullptr; }
  m->version = ~0ull;
}

void mg_destroy(kf_problem *p) {
  if (!p || !p->mg) return;
  mg_free_fields(p->mg);
  delete p->mg;
  p->mg = nullptr;
}

template <typename T> static kf_status mg_alloc(T **q, size_t bytes) {
  if (kf_malloc((void **)q, bytes ? bytes : 1) != hipSuccess) {
    *q = nullptr;
    set_error("multigrid: hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return KF_ENOMEM;
  }
  return KF_OK;
}

// levels, fields and the factorised coarsest problem for the problem's current gamma
static kf_status mg_build(kf_problem *p) {
  MgState *m = p->mg;
  if (m->version == p->gamma_version && !m->lev.empty()) return KF_OK;
  mg_free_fields(m);
  const size_t K = p->K, es = fsz(m);
  // level sizes
  int nx = p->nx, nz = p->nz, npml = p->npml;
  double h = p->h;
  for (;;) {
    MgLevel L;
    L.nx = nx; L.nz = nz; L.npml = npml; L.h = h;
    m->lev.push_back(L);
    if (nx % 2 == 0 || nz % 2 == 0 || std::min(nx, nz) < m->n_min || m->lev.size() == 8) break;
    nx = (nx + 1) / 2; nz = (nz + 1) / 2; h *= 2.0; npml /= 2;
  }
  if (m->lev.size() < 2) {
    m->lev.clear();
    set_error("multigrid: the grid admits no coarser level (both sizes must be odd and at least n_min)");
    return KF_ESHAPE;
  }
  // level 0 shares the problem's arrays; the others own theirs
  m->lev[0].gamma = p->gamma;
  m->lev[0].xn = p->xn; m->lev[0].ixh = p->ixh; m->lev[0].zn = p->zn; m->lev[0].izh = p->izh;
  for (size_t l = 1; l < m->lev.size(); ++l) {
    MgLevel &L = m->lev[l], &F = m->lev[l - 1];
    CHECK_ST(mg_alloc(&L.gamma, sizeof(double) * L.nx * L.nz));
    CHECK_ST(mg_alloc(&L.xn, sizeof(double2) * L.nx)); CHECK_ST(mg_alloc(&L.ixh, sizeof(double2) * (L.nx + 1)));
    CHECK_ST(mg_alloc(&L.zn, sizeof(double2) * L.nz)); CHECK_ST(mg_alloc(&L.izh, sizeof(double2) * (L.nz + 1)));
    hipLaunchKernelGGL(k_mg_inject, dim3((L.nx * L.nz + 255) / 256), dim3(256), 0, p->stream, F.nx, L.nx, L.nz,
                       (const double *)F.gamma, L.gamma);
    LAUNCH_CHECK();
    CHECK_ST(launch_stretch(p->stream, L.nx, L.h, L.npml, p->omega, p->d.pml_r0, p->d.pml_cref, L.xn, L.ixh));
    CHECK_ST(launch_stretch(p->stream, L.nz, L.h, L.npml, p->omega, p->d.pml_r0, p->d.pml_cref, L.zn, L.izh));
  }
  for (size_t l = 0; l + 1 < m->lev.size(); ++l) {
    MgLevel &L = m->lev[l];
    const size_t bytes = es * K * L.nx * L.nz;
    for (void **q : {&L.b, &L.xa, &L.xb, &L.r, &L.cp}) CHECK_ST(mg_alloc(q, bytes));
  }
  {   // the coarsest level's right-hand side and solution
    MgLevel &L = m->lev.back();
    const size_t bytes = es * K * L.nx * L.nz;
    CHECK_ST(mg_alloc(&L.b, bytes));
    CHECK_ST(mg_alloc(&L.xa, bytes));
  }
  // the coarsest level as a problem of its own, with the shift, factorised now
  {
    MgLevel &L = m->lev.back();
    kf_desc d = p->d;
    d.nx = L.nx; d.nz = L.nz; d.h = L.h; d.npml = L.npml;
    std::vector<int32_t> zero((size_t)p->K, 0);
    int32_t r0 = 0;
    d.src_ix = zero.data(); d.src_iz = zero.data();
    d.nrec = 1; d.rec_ix = &r0; d.rec_iz = &r0; d.w = nullptr;
    HIP_TRY(hipStreamSynchronize(p->stream));
    CHECK_ST(kf_create(&d, L.gamma, 1, p->stream, &m->coarse));
    m->coarse->beta = m->beta;
    CHECK_ST(blu_factor(m->coarse, m->prec == KF_C64 ? 3 : 1));
  }
  const size_t n0 = K * p->Nu;
  for (void *&q : m->bf) CHECK_ST(mg_alloc(&q, es * n0));
  CHECK_ST(mg_alloc(&m->partial, sizeof(double) * 2 * K * DB * 2));
  CHECK_ST(mg_alloc(&m->dots, sizeof(double2) * 2 * K));
  CHECK_ST(mg_alloc(&m->sc, sizeof(double2) * 6 * K));
  if (hipHostMalloc((void **)&m->host, sizeof(double) * K) != hipSuccess) {
    m->host = nullptr;
    set_error("multigrid: hipHostMalloc failed");
    return KF_ENOMEM;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  m->version = p->gamma_version;
  return KF_OK;
}

// x-line sweep: parallel cyclic reduction in LDS for rows of up to PCR_MAX nodes, the
// thread-per-row Thomas kernel for longer ones
template <typename R>
static kf_status xline(hipStream_t s, const Grid &g, int K, const cplx<R> *x, const cplx<R> *b, cplx<R> *y,
                       cplx<R> *cp) {
  if (g.nx <= PCR_MAX) {
    const size_t lds = 4 * sizeof(cplx<R>) * (size_t)g.nx;
    static bool attr_set = false;
    if (!attr_set) {
      HIP_TRY(hipFuncSetAttribute((const void *)k_mg_xline_pcr<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(4 * sizeof(cplx<R>) * PCR_MAX)));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_mg_xline_pcr<R>, dim3((unsigned)(K * g.nz)), dim3(PCR_T), lds, s, g, K, x, b, y);
  } else {
    hipLaunchKernelGGL(k_mg_xline<R>, dim3(nblk((size_t)K * g.nz)), dim3(TB), 0, s, g, K, x, b, y, cp);
  }
  LAUNCH_CHECK();
  return KF_OK;
}

// ---------------------------------------------------------------------------
// V-cycle: x = V(b) on level l (b and x are that level's R fields)
// ---------------------------------------------------------------------------
template <typename R>
static kf_status vcycle(kf_problem *p, size_t l, const cplx<R> *b, cplx<R> *x) {
  MgState *m = p->mg;
  MgLevel &L = m->lev[l];
  const int K = p->K;
  hipStream_t s = p->stream;
  if (l + 1 == m->lev.size()) return blu_solve<R>(m->coarse, 0, b, x);
  const Grid g = L.grid(p->omega, m->beta);
  const size_t n = (size_t)K * L.nx * L.nz;
  cplx<R> *xa = x, *xb = (cplx<R> *)L.xb, *r = (cplx<R> *)L.r, *cp = (cplx<R> *)L.cp;
  const unsigned gz = nblk((size_t)K * L.nx), gx = nblk((size_t)K * L.nz);
  // pre-smoothing from x = 0: z-lines (into xb), x-lines (into xa)
  hipLaunchKernelGGL(k_mg_zline<R>, dim3(gz), dim3(TB), 0, s, g, K, (const cplx<R> *)nullptr, b, xb, cp);
  LAUNCH_CHECK();
  CHECK_ST(xline<R>(s, g, K, xb, b, xa, cp));
  // coarse-grid correction
  hipLaunchKernelGGL(k_mg_residual<R>, dim3(nblk(n)), dim3(TB), 0, s, g, K, (const cplx<R> *)xa, b, r);
  LAUNCH_CHECK();
  MgLevel &C = m->lev[l + 1];
  hipLaunchKernelGGL(k_mg_restrict<R>, dim3(nblk((size_t)K * C.nx * C.nz)), dim3(TB), 0, s, K, L.nx, L.nz, C.nx,
                     C.nz, (const cplx<R> *)r, (cplx<R> *)C.b);
  LAUNCH_CHECK();
  CHECK_ST(vcycle<R>(p, l + 1, (const cplx<R> *)C.b, (cplx<R> *)C.xa));
  hipLaunchKernelGGL(k_mg_prolong_add<R>, dim3(nblk(n)), dim3(TB), 0, s, K, L.nx, L.nz, C.nx, C.nz,
                     (const cplx<R> *)C.xa, xa);
  LAUNCH_CHECK();
  // post-smoothing: x-lines (into xb), z-lines (into xa)
  CHECK_ST(xline<R>(s, g, K, xa, b, xb, cp));
  hipLaunchKernelGGL(k_mg_zline<R>, dim3(gz), dim3(TB), 0, s, g, K, (const cplx<R> *)xb, b, xa, cp);
  LAUNCH_CHECK();
  return KF_OK;
}

// per-source (a, b) into dots[0..K)
template <typename R>
static kf_status src_dots(kf_problem *p, const cplx<R> *a, const cplx<R> *b, double2 *out, double *partial) {
  hipLaunchKernelGGL(k_src_dot<R>, dim3(DB, p->K), dim3(TB), 0, p->stream, (size_t)p->Nu, a, b, partial);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_src_dot_finish, dim3((p->K + 63) / 64), dim3(64), 0, p->stream, p->K, partial, out);
  LAUNCH_CHECK();
  return KF_OK;
}

// y = A x in R (the unshifted operator of the problem)
template <typename R> static kf_status apply_A(kf_problem *p, const cplx<R> *x, cplx<R> *y) {
  return launch_stencil<R>(p, 0, x, y);
}

// BiCGStab for A x = b (c128 b, x; the adjoint through conjugation), right-preconditioned
// by one V-cycle; stops when every source meets ||b_k - A x_k|| <= rtol ||b_k||.
template <typename R>
static kf_status mg_bicgstab(kf_problem *p, int adjoint, const double2 *b, double2 *x, double rtol, int maxit,
                             kf_mg_stats *st) {
  MgState *m = p->mg;
  const int K = p->K;
  const size_t n = (size_t)K * p->Nu;
  hipStream_t s = p->stream;
  cplx<R> *X = (cplx<R> *)m->bf[0], *Rr = (cplx<R> *)m->bf[1], *Rh = (cplx<R> *)m->bf[2], *P = (cplx<R> *)m->bf[3],
          *V = (cplx<R> *)m->bf[4], *S = (cplx<R> *)m->bf[5], *T = (cplx<R> *)m->bf[6], *PH = (cplx<R> *)m->bf[7],
          *SH = (cplx<R> *)m->bf[8];
  const unsigned gb = nblk(n);
  // r = b (x = 0), rhat = r, p = v = 0, per-source scalars rho = alpha = omega = 1, active
  hipLaunchKernelGGL(k_mg_in<R>, dim3(std::min<size_t>(gb, 8192)), dim3(TB), 0, s, (int64_t)n, adjoint, b, Rr);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(Rh, Rr, sizeof(cplx<R>) * n, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemsetAsync(X, 0, sizeof(cplx<R>) * n, s));
  HIP_TRY(hipMemsetAsync(P, 0, sizeof(cplx<R>) * n, s));
  HIP_TRY(hipMemsetAsync(V, 0, sizeof(cplx<R>) * n, s));
  std::vector<double2> init((size_t)6 * K);
  for (int k = 0; k < K; ++k) {
    double2 *q = init.data() + (size_t)6 * k;
    q[0] = q[1] = q[2] = make_double2(1.0, 0.0);
    q[3] = q[4] = make_double2(0.0, 0.0);
    q[5] = make_double2(1.0, 0.0);
  }
  HIP_TRY(hipMemcpyAsync(m->sc, init.data(), sizeof(double2) * 6 * K, hipMemcpyHostToDevice, s));
  // ||b_k||
  std::vector<double> bn(K), rn(K);
  CHECK_ST(src_dots<R>(p, Rr, Rr, m->dots, m->partial));
  std::vector<double2> hd(K);
  HIP_TRY(hipMemcpyAsync(hd.data(), m->dots, sizeof(double2) * K, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < K; ++k) bn[k] = std::sqrt(std::max(hd[k].x, 0.0));
  std::vector<char> active(K, 1);
  for (int k = 0; k < K; ++k)
    if (bn[k] == 0.0) active[k] = 0;
  static const double2 zero2 = {0.0, 0.0};
  auto deactivate = [&](int k) -> kf_status {
    HIP_TRY(hipMemcpyAsync(m->sc + (size_t)6 * k + 5, &zero2, sizeof(double2), hipMemcpyHostToDevice, s));
    return KF_OK;
  };
  for (int k = 0; k < K; ++k)
    if (!active[k]) CHECK_ST(deactivate(k));
  int it = 0, vcycles = 0;
  double worst = 0.0;
  kf_status status = KF_OK;
  double2 *d0 = m->dots, *d1 = m->dots + K;
  double *part0 = m->partial, *part1 = m->partial + (size_t)K * DB * 2;
  for (;;) {
    bool any = false;
    for (int k = 0; k < K; ++k) any = any || active[k];
    if (!any) break;
    if (it >= maxit) { status = KF_ENOCONV; break; }
    // rho_new, beta; p = r + beta (p - omega v); ph = V(p); v = A ph; alpha
    CHECK_ST(src_dots<R>(p, Rh, Rr, d0, part0));
    hipLaunchKernelGGL(k_bicg_scalars, dim3((K + 63) / 64), dim3(64), 0, s, K, 0, (const double2 *)d0,
                       (const double2 *)d1, m->sc);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bicg_update<R>, dim3(gb), dim3(TB), 0, s, 0, (size_t)p->Nu, K, (const double2 *)m->sc, P, Rr,
                       V, (cplx<R> *)nullptr, (cplx<R> *)nullptr, (cplx<R> *)nullptr);
    LAUNCH_CHECK();
    CHECK_ST(vcycle<R>(p, 0, P, PH));
    CHECK_ST(apply_A<R>(p, PH, V));
    CHECK_ST(src_dots<R>(p, Rh, V, d0, part0));
    hipLaunchKernelGGL(k_bicg_scalars, dim3((K + 63) / 64), dim3(64), 0, s, K, 1, (const double2 *)d0,
                       (const double2 *)d1, m->sc);
    LAUNCH_CHECK();
    // s = r - alpha v; sh = V(s); t = A sh; omega
    hipLaunchKernelGGL(k_bicg_update<R>, dim3(gb), dim3(TB), 0, s, 1, (size_t)p->Nu, K, (const double2 *)m->sc, S, Rr,
                       V, (cplx<R> *)nullptr, (cplx<R> *)nullptr, (cplx<R> *)nullptr);
    LAUNCH_CHECK();
    CHECK_ST(vcycle<R>(p, 0, S, SH));
    CHECK_ST(apply_A<R>(p, SH, T));
    CHECK_ST(src_dots<R>(p, T, S, d0, part0));
    CHECK_ST(src_dots<R>(p, T, T, d1, part1));
    hipLaunchKernelGGL(k_bicg_scalars, dim3((K + 63) / 64), dim3(64), 0, s, K, 2, (const double2 *)d0,
                       (const double2 *)d1, m->sc);
    LAUNCH_CHECK();
    // x += alpha ph + omega sh; r = s - omega t
    hipLaunchKernelGGL(k_bicg_update<R>, dim3(gb), dim3(TB), 0, s, 2, (size_t)p->Nu, K, (const double2 *)m->sc, X, PH,
                       SH, Rr, S, T);
    LAUNCH_CHECK();
    vcycles += 2;
    ++it;
    // residual norms (the recurrence's r), one host round trip per iteration
    CHECK_ST(src_dots<R>(p, Rr, Rr, d0, part0));
    HIP_TRY(hipMemcpyAsync(hd.data(), d0, sizeof(double2) * K, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    worst = 0.0;
    for (int k = 0; k < K; ++k) {
      if (!active[k]) continue;
      const double rel = std::sqrt(std::max(hd[k].x, 0.0)) / bn[k];
      if (!std::isfinite(rel)) { status = KF_ENAN; break; }
      if (rel <= rtol) { active[k] = 0; CHECK_ST(deactivate(k)); }
      worst = std::max(worst, rel);
    }
    if (status != KF_OK) break;
  }
  // x out (c128), conjugated back for the adjoint
  hipLaunchKernelGGL(k_mg_out<R>, dim3(std::min<size_t>(gb, 8192)), dim3(TB), 0, s, (int64_t)n, adjoint,
                     (const cplx<R> *)X, x);
  LAUNCH_CHECK();
  if (st) { st->iters = it; st->vcycles = vcycles; st->rel_res_max = -1.0; }
  if (status == KF_ENAN) { set_error("multigrid BiCGStab: non-finite residual"); return KF_ENAN; }
  if (status == KF_ENOCONV) set_error("multigrid BiCGStab reached maxit");
  return status;
}

// ---------------------------------------------------------------------------
// entry points used by api.hip
// ---------------------------------------------------------------------------
kf_status mg_configure(kf_problem *p, int prec, double beta, double rtol, int maxit, int n_min) {
  if (prec != KF_C64 && prec != KF_C128) { set_error("multigrid precision must be KF_C64 or KF_C128"); return KF_EINVAL; }
  if (!(beta > 0.0) || !std::isfinite(beta)) { set_error("beta must be > 0"); return KF_EINVAL; }
  if (!(rtol > 0.0 && rtol < 1.0)) { set_error("inner rtol must be in (0, 1)"); return KF_EINVAL; }
  if (maxit < 1) { set_error("inner maxit must be >= 1"); return KF_EINVAL; }
  if (n_min < 3) { set_error("n_min must be >= 3"); return KF_EINVAL; }
  if (!p->mg) p->mg = new MgState();
  MgState *m = p->mg;
  if (m->prec != prec || m->beta != beta || m->n_min != n_min) mg_free_fields(m);
  m->prec = prec; m->beta = beta; m->rtol = rtol; m->maxit = maxit; m->n_min = n_min;
  return KF_OK;
}

kf_status mg_solve(kf_problem *p, int adjoint, const double2 *b, double2 *x, double rtol, int maxit, kf_mg_stats *st) {
  if (!p->mg) CHECK_ST(mg_configure(p, KF_C64, 0.5, 1e-3, 200, 20));
  CHECK_ST(mg_build(p));
  if (rtol <= 0.0) rtol = p->mg->rtol;
  if (maxit <= 0) maxit = p->mg->maxit;
  ProfScope ps(p, PROF_MG);
  return p->mg->prec == KF_C64 ? mg_bicgstab<float>(p, adjoint, b, x, rtol, maxit, st)
                               : mg_bicgstab<double>(p, adjoint, b, x, rtol, maxit, st);
}

kf_status mg_vcycle_apply(kf_problem *p, const double2 *b, double2 *x) {
  if (!p->mg) CHECK_ST(mg_configure(p, KF_C64, 0.5, 1e-3, 200, 20));
  CHECK_ST(mg_build(p));
  MgState *m = p->mg;
  const size_t n = (size_t)p->K * p->Nu;
  const unsigned gb = std::min<size_t>(nblk(n), 8192);
  if (m->prec == KF_C64) {
    float2 *B = (float2 *)m->bf[1], *X = (float2 *)m->bf[0];
    hipLaunchKernelGGL(k_mg_in<float>, dim3(gb), dim3(TB), 0, p->stream, (int64_t)n, 0, b, B);
    LAUNCH_CHECK();
    CHECK_ST(vcycle<float>(p, 0, B, X));
    hipLaunchKernelGGL(k_mg_out<float>, dim3(gb), dim3(TB), 0, p->stream, (int64_t)n, 0, (const float2 *)X, x);
    LAUNCH_CHECK();
  } else {
    double2 *B = (double2 *)m->bf[1], *X = (double2 *)m->bf[0];
    hipLaunchKernelGGL(k_mg_in<double>, dim3(gb), dim3(TB), 0, p->stream, (int64_t)n, 0, b, B);
    LAUNCH_CHECK();
    CHECK_ST(vcycle<double>(p, 0, B, X));
    hipLaunchKernelGGL(k_mg_out<double>, dim3(gb), dim3(TB), 0, p->stream, (int64_t)n, 0, (const double2 *)X, x);
    LAUNCH_CHECK();
  }
  return KF_OK;
}

int mg_levels(kf_problem *p, int *dims /*[host][2 * 8] or NULL*/) {
  if (!p->mg || p->mg->lev.empty()) return 0;
  if (dims)
    for (size_t l = 0; l < p->mg->lev.size() && l < 8; ++l) {
      dims[2 * l] = p->mg->lev[l].nx;
      dims[2 * l + 1] = p->mg->lev[l].nz;
    }
  return (int)p->mg->lev.size();
}
