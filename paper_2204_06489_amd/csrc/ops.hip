// Field kernels of the full-space Gauss-Newton step on gfx950 (wave64).
//
// Layout: fields [K][nz][nx] (x fastest), control [nzc][nxc] on the core nodes,
// packed KKT vectors [du (K*Nu) | ds (Ng) | lambda (K*Nu)].
// All kernels are memory-bound stencil / elementwise sweeps; none is a dense
// contraction, so none uses MFMA.
#include "common.h"

#include <cmath>
#include <mutex>

namespace {

constexpr int BX = 64;   // one wavefront across x
constexpr int BY = 4;    // four wavefronts down z

// ---------------------------------------------------------------------------
// PML stretch factors (Section 2; quadratic profile with design reflection r0)
// ---------------------------------------------------------------------------
__global__ void k_stretch(int n, double h, int npml, double omega, double r0, double cref,
                          double2 *fn, double2 *ifh) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n) return;
  double width = npml * h;
  auto sigma = [&](double x) {
    if (npml == 0) return 0.0;
    double smax = 3.0 * cref / (2.0 * width) * log(1.0 / r0);
    double d = fmax(fmax(npml * h - x, x - (n - 1 - npml) * h), 0.0);
    return smax * (d / width) * (d / width);
  };
  if (t < n) fn[t] = make_double2(1.0, sigma(t * h) / omega);
  // face t sits at (t - 1/2) h
  double2 f = make_double2(1.0, sigma((t - 0.5) * h) / omega);
  ifh[t] = cdiv(make_double2(1.0, 0.0), f);
}

// Stores that are not read again by the same kernel: the non-temporal hint keeps the
// output lines from displacing the lambda / du rows that neighbouring workgroups still
// read through L2.
typedef double kf_dv2 __attribute__((ext_vector_type(2)));
__device__ inline void store_stream(double2 *q, double2 v) {
  const kf_dv2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, (kf_dv2 *)q);
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD b mod 8).
// Renumber them so that XCD x owns one contiguous run of logical workgroups.
__device__ inline unsigned xcd_contiguous(unsigned b, unsigned n) {
  const unsigned x = b & 7, s = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + s;
}

// Fused KKT matvec (eq. KKT with the blocks of eq. partitioned_system_matrix).
// Logical workgroup L = chunk + chunks * group owns the KKT_WG consecutive nodes
// [chunk * KKT_WG, ...) of the flattened grid, one per thread, and loops over the
// sources of its group.  Each node reads lambda_k and du_k at itself and its four
// neighbours (the x-neighbours from the adjacent lanes, the z-neighbours from the rows
// above and below, read by the workgroups of those rows too), u_k at itself, and
// writes y_u,k = A^H lambda_k and y_lambda,k = A du_k - P_k ds.  Because each XCD
// owns a contiguous run of chunks and all workgroups of a group walk the same sources
// in the same order, the neighbour rows are mostly L2 hits.  The loop is unrolled by
// two so that two sources' loads are in flight.  With one group the control row
// y_s = eps ds - sum_k P_k^* lambda_k is written here; otherwise each group writes
// its part of the sum over k into ys_part ([group][Ng]) and k_kkt_ys_finish adds the
// groups in fixed order.
// The value held by the previous (UP) or the next lane of the wavefront, by DPP wave
// shifts (wave_shr:1 / wave_shl:1); the first (last) lane receives zero.  Consecutive
// lanes hold consecutive nodes of the flattened grid, so a node's x-neighbours come
// from the adjacent lanes instead of loads.
template <bool UP> __device__ __forceinline__ int wave_shift(int v) {
  return __builtin_amdgcn_update_dpp(0, v, UP ? 0x138 : 0x130, 0xf, 0xf, false);
}
template <bool UP> __device__ __forceinline__ double wave_shift(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = wave_shift<UP>((int)b), hi = wave_shift<UP>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <bool UP> __device__ __forceinline__ float wave_shift(float v) {
  return __builtin_bit_cast(float, wave_shift<UP>(__builtin_bit_cast(int, v)));
}
template <bool UP> __device__ __forceinline__ double2 wave_shift(double2 v) {
  return make_double2(wave_shift<UP>(v.x), wave_shift<UP>(v.y));
}
template <bool UP> __device__ __forceinline__ float2 wave_shift(float2 v) {
  return make_float2(wave_shift<UP>(v.x), wave_shift<UP>(v.y));
}
constexpr int KKT_WG = 256;
__global__ __launch_bounds__(KKT_WG) void k_kkt_apply(Grid g, int K, int kpg, int nxc, unsigned chunks,
                                                      double eps, const double2 *__restrict__ xi,
                                                      const double2 *__restrict__ un,
                                                      double2 *__restrict__ y, double2 *__restrict__ ys_part) {
  const unsigned L = xcd_contiguous(blockIdx.x, gridDim.x);
  const unsigned chunk = L % chunks, grp = L / chunks;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t p = (size_t)chunk * KKT_WG + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if (p >= Nu) return;
  const int j = (int)(p / g.nx), i = (int)(p - (size_t)j * g.nx);
  const int nzc = g.nz - 2 * g.npml;
  const size_t Ng = (size_t)nxc * nzc;
  const double2 *du = xi;
  const double2 *dsv = xi + (size_t)K * Nu;
  const double2 *lam = dsv + Ng;
  double2 *yu = y;
  double2 *yl = y + (size_t)K * Nu + Ng;
  const double w2 = g.omega * g.omega;
  const bool hxm = i > 0, hxp = i + 1 < g.nx, hzm = j > 0, hzp = j + 1 < g.nz;
  const Stencil5 s = stencil_at(g, i, j);
  const bool core = i >= g.npml && i < g.nx - g.npml && j >= g.npml && j < g.nz - g.npml;
  const size_t c = core ? (size_t)(j - g.npml) * nxc + (i - g.npml) : 0;
  const double2 ds = core ? dsv[c] : make_double2(0.0, 0.0);
  const double2 w2ds = cscale(ds, w2);
  double2 acc = make_double2(0.0, 0.0);
  const int k0 = grp * kpg, k1 = min(K, k0 + kpg);
  auto source = [&](int k) {
    const size_t o = (size_t)k * Nu + p;
    const double2 l0 = lam[o], d0 = du[o], u = un[o];
    double2 ah = cmulc(s.cc, l0);     // conj(weight) * lambda: A^H lambda
    double2 a = cmul(s.cc, d0);
    // x-neighbours from the adjacent lanes, the wavefront's end lanes from memory (every
    // lane runs the shifts: the branches below only pick the terms)
    double2 lm = wave_shift<true>(l0), dm = wave_shift<true>(d0), lp = wave_shift<false>(l0), dp = wave_shift<false>(d0);
    if (lane == 0 && hxm) { lm = lam[o - 1]; dm = du[o - 1]; }
    if (lane == 63 && hxp) { lp = lam[o + 1]; dp = du[o + 1]; }
    if (hxm) { ah = cadd(ah, cmulc(s.cxm, lm)); cfma(a, s.cxm, dm); }
    if (hxp) { ah = cadd(ah, cmulc(s.cxp, lp)); cfma(a, s.cxp, dp); }
    if (hzm) { ah = cadd(ah, cmulc(s.czm, lam[o - g.nx])); cfma(a, s.czm, du[o - g.nx]); }
    if (hzp) { ah = cadd(ah, cmulc(s.czp, lam[o + g.nx])); cfma(a, s.czp, du[o + g.nx]); }
    store_stream(yu + o, ah);
    store_stream(yl + o, csub(a, cmul(u, w2ds)));
    acc = cadd(acc, cmulc(u, l0));
  };
  // two sources per pass (their loads in flight together; the trip count is uniform, so
  // every lane runs the wave shifts of both)
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    source(k);
    source(k + 1);
  }
  if (k < k1) source(k);
  if (!core) return;
  if (gridDim.x == chunks)
    y[(size_t)K * Nu + c] = csub(cscale(ds, eps), cscale(acc, w2));
  else
    ys_part[(size_t)grp * Ng + c] = acc;
}

__device__ inline void store_stream(float2 *q, float2 v) {
  typedef float kf_fv2 __attribute__((ext_vector_type(2)));
  const kf_fv2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, (kf_fv2 *)q);
}

// y_k = A x_k, or A^H x_k (the conjugate weights: A is complex symmetric), for all
// sources (eq. Au=f).  Laid out like k_kkt_apply: logical workgroup chunk + chunks *
// group owns KKT_WG consecutive nodes of the flattened grid and the STEN_KPG sources
// of its group, the XCDs each own a contiguous run of chunks (neighbour rows are L2
// hits, x-neighbours come from the adjacent lanes), the source loop is unrolled by two
// and the outputs are streamed.
constexpr int STEN_KPG = 8;
template <typename R, bool ADJ>
__global__ __launch_bounds__(KKT_WG) void k_stencil(Grid g, int K, unsigned chunks, const cplx<R> *__restrict__ x,
                                                    cplx<R> *__restrict__ y) {
  const unsigned L = xcd_contiguous(blockIdx.x, gridDim.x);
  const unsigned chunk = L % chunks, grp = L / chunks;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t p = (size_t)chunk * KKT_WG + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if (p >= Nu) return;
  const int j = (int)(p / g.nx), i = (int)(p - (size_t)j * g.nx);
  Stencil5 s = stencil_at(g, i, j);
  if (ADJ) { s.cc = cconj(s.cc); s.cxm = cconj(s.cxm); s.cxp = cconj(s.cxp); s.czm = cconj(s.czm); s.czp = cconj(s.czp); }
  const cplx<R> cc = ccast<R>(s.cc), cxm = ccast<R>(s.cxm), cxp = ccast<R>(s.cxp),
                czm = ccast<R>(s.czm), czp = ccast<R>(s.czp);
  const bool hxm = i > 0, hxp = i + 1 < g.nx, hzm = j > 0, hzp = j + 1 < g.nz;
  const int k0 = grp * STEN_KPG, k1 = min(K, k0 + STEN_KPG);
  auto source = [&](int k) {
    const cplx<R> *xk = x + (size_t)k * Nu;
    const cplx<R> xc = xk[p];
    cplx<R> xm = wave_shift<true>(xc), xp = wave_shift<false>(xc);   // x-neighbours from the adjacent lanes
    if (lane == 0 && hxm) xm = xk[p - 1];
    if (lane == 63 && hxp) xp = xk[p + 1];
    cplx<R> acc = cmul(cc, xc);
    if (hxm) cfma(acc, cxm, xm);
    if (hxp) cfma(acc, cxp, xp);
    if (hzm) cfma(acc, czm, xk[p - g.nx]);
    if (hzp) cfma(acc, czp, xk[p + g.nx]);
    store_stream(y + (size_t)k * Nu + p, acc);
  };
  int k = k0;   // two sources per pass, as in k_kkt_apply
  for (; k + 1 < k1; k += 2) {
    source(k);
    source(k + 1);
  }
  if (k < k1) source(k);
}

// y_s = eps ds - omega^2 sum over source groups (fixed order)
__global__ void k_kkt_ys_finish(size_t Ng, int groups, double eps, double w2, const double2 *__restrict__ ds,
                                const double2 *__restrict__ part, double2 *__restrict__ ys) {
  size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Ng) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = 0; q < groups; ++q) acc = cadd(acc, part[(size_t)q * Ng + c]);
  ys[c] = csub(cscale(ds[c], eps), cscale(acc, w2));
}

// y_u,k(node) += (sum of W_k^2 over the receivers at that node) du_k(node)
__global__ void k_kkt_F(int K, int nru, const int32_t *__restrict__ rnode, const double *__restrict__ wsq,
                        size_t Nu, const double2 *__restrict__ du, double2 *__restrict__ yu) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * nru) return;
  int k = t / nru, u = t % nru;
  size_t o = (size_t)k * Nu + rnode[u];
  double2 v = yu[o];
  cfma(v, make_double2(wsq[t], 0.0), du[o]);
  yu[o] = v;
}

// ---------------------------------------------------------------------------
// Preconditioner stage 2 (eq. precond, middle row) fused with the right-hand side
// of stage 3:
//   z_s   = (y_s + omega^2 sum_k E^T (conj(u_k) z_lam,k)) / eps
//   rhs_k = y_lam,k + omega^2 u_k (E z_s)            -> written into z_u,k
// A workgroup takes 64 consecutive nodes of the flattened grid; its S2_G rows of
// threads split the sources (thread row r takes k = r, r + S2_G, ...), so S2_G times
// as many loads are in flight as with one thread per node.  The rows' parts of the
// sum over k are added in fixed order through LDS.
// ---------------------------------------------------------------------------
constexpr int S2_G = 4;
__global__ __launch_bounds__(64 * S2_G) void k_precond_stage2(Grid g, int K, int nxc, double eps,
                                                             const double2 *__restrict__ y,
                                                             const double2 *__restrict__ un,
                                                             double2 *__restrict__ z) {
  __shared__ double2 part[S2_G][64];
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t p = (size_t)blockIdx.x * 64 + threadIdx.x;
  const int r = threadIdx.y;
  const bool valid = p < Nu;
  const int j = valid ? (int)(p / g.nx) : 0, i = valid ? (int)(p - (size_t)j * g.nx) : 0;
  const int nzc = g.nz - 2 * g.npml;
  const size_t Ng = (size_t)nxc * nzc;
  const bool core = valid && i >= g.npml && i < g.nx - g.npml && j >= g.npml && j < g.nz - g.npml;
  const size_t c = core ? (size_t)(j - g.npml) * nxc + (i - g.npml) : 0;
  const double2 *ys = y + (size_t)K * Nu;
  const double2 *yl = ys + Ng;
  double2 *zu = z;
  double2 *zs = z + (size_t)K * Nu;
  const double2 *zl = zs + Ng;
  const double w2 = g.omega * g.omega;
  double2 acc = make_double2(0.0, 0.0);
  if (core) {
#pragma unroll 4
    for (int k = r; k < K; k += S2_G) {
      const size_t o = (size_t)k * Nu + p;
      acc = cadd(acc, cmulc(un[o], zl[o]));
    }
  }
  part[r][threadIdx.x] = acc;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (core) {
    double2 sum = part[0][threadIdx.x];
#pragma unroll
    for (int q = 1; q < S2_G; ++q) sum = cadd(sum, part[q][threadIdx.x]);
    s = cscale(cadd(ys[c], cscale(sum, w2)), 1.0 / eps);
    if (r == 0) zs[c] = s;
  }
  if (!valid) return;
  const double2 w2s = cscale(s, w2);
#pragma unroll 4
  for (int k = r; k < K; k += S2_G) {
    const size_t o = (size_t)k * Nu + p;
    zu[o] = cadd(yl[o], cmul(un[o], w2s));
  }
}

// ---------------------------------------------------------------------------

// f_k = e_src_k / h^2
__global__ void k_sources(int K, size_t Nu, const int32_t *__restrict__ src, double val, double2 *f) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)K * Nu) return;
  int k = (int)(t / Nu);
  size_t p = t % Nu;
  f[t] = make_double2(p == (size_t)src[k] ? val : 0.0, 0.0);
}

// r_k = d_k - Q u_k,  wr = W r  (per receiver)
__global__ void k_residual(int K, int nrec, size_t Nu, const int32_t *__restrict__ rec,
                           const double *__restrict__ w, const double2 *__restrict__ d,
                           const double2 *__restrict__ u, double2 *r, double2 *wr) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * nrec) return;
  int k = t / nrec, q = t % nrec;
  double2 v = csub(d[t], u[(size_t)k * Nu + rec[q]]);
  r[t] = v;
  wr[t] = cscale(v, w[t]);
}

// b_u,k(node) = sum over receivers at the node of W_k^2 r_k   (Q^T W^T W r, eq. KKT)
__global__ void k_rhs_u(int K, int nru, int nrec, size_t Nu, const int32_t *__restrict__ rnode,
                        const int32_t *__restrict__ rptr, const int32_t *__restrict__ rlist,
                        const double *__restrict__ w, const double2 *__restrict__ r, double2 *bu) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * nru) return;
  int k = t / nru, u = t % nru;
  double2 acc = make_double2(0.0, 0.0);
  for (int e = rptr[u]; e < rptr[u + 1]; ++e) {
    int q = rlist[e];
    double ww = w[k * nrec + q];
    acc = cadd(acc, cscale(r[k * nrec + q], ww * ww));
  }
  bu[(size_t)k * Nu + rnode[u]] = acc;
}

// b_s = -eps s_n on the control nodes
__global__ void k_rhs_s(int nx, int npml, int nxc, int nzc, double eps, const double *__restrict__ gamma,
                        double2 *bs) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxc * nzc) return;
  int ic = t % nxc, jc = t / nxc;
  bs[t] = make_double2(-eps * gamma[(size_t)(jc + npml) * nx + ic + npml], 0.0);
}

// gamma_core += Re(ds)   (s_{n+1} = s_n + ds, Section 3)
__global__ void k_update_gamma(int nx, int npml, int nxc, int nzc, const double2 *__restrict__ ds,
                               double *gamma) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxc * nzc) return;
  int ic = t % nxc, jc = t / nxc;
  gamma[(size_t)(jc + npml) * nx + ic + npml] += ds[t].x;
}

// grad[j][i] = omega^2 sum_k Re(conj(mu_k) X_i Z_j u_k)
template <typename C>
__global__ __launch_bounds__(BX *BY) void k_grad_gamma(Grid g, int K, const C *__restrict__ u,
                                                        const C *__restrict__ mu, double *grad) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.nz) return;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t p = (size_t)j * g.nx + i;
  const double2 xz = cmul(g.xn[i], g.zn[j]);
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    C a = u[k * Nu + p], m = mu[k * Nu + p];
    double2 ud = make_double2((double)a.x, (double)a.y);
    double2 md = make_double2((double)m.x, (double)m.y);
    acc += cmulc(md, cmul(xz, ud)).x;
  }
  grad[p] = g.omega * g.omega * acc;
}

__global__ void k_axpy(int64_t n, double2 a, const double2 *__restrict__ x, double2 *y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < n; t += (int64_t)gridDim.x * blockDim.x) y[t] = cadd(y[t], cmul(a, x[t]));
}
// y = a x + b y
__global__ void k_axpby(int64_t n, double2 a, const double2 *__restrict__ x, double2 b, double2 *y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < n; t += (int64_t)gridDim.x * blockDim.x) y[t] = cadd(cmul(a, x[t]), cmul(b, y[t]));
}

// ---------------------------------------------------------------------------
// Pieces of the reduced Hessian product of Section 3,
//   H v = eps v + sum_k J_k^* W_k^2 J_k v,   J_k = Q A^-1 P_k,  P_k = omega^2 diag(u_k) E:
// P v for every source (the right-hand sides of the forward solves), Q^T W^2 Q on the
// solved fields, and eps v + P^* lambda (the sum over sources of the adjoint fields).
// ---------------------------------------------------------------------------
// out_k(node) = omega^2 u_k(node) v(core index of node), 0 in the PML
__global__ void k_scatter_P(Grid g, int K, int nxc, const double2 *__restrict__ un, const double2 *__restrict__ v,
                            double2 *__restrict__ out) {
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)K * Nu) return;
  const size_t p = t % Nu;
  const int j = (int)(p / g.nx), i = (int)(p - (size_t)j * g.nx);
  const bool core = i >= g.npml && i < g.nx - g.npml && j >= g.npml && j < g.nz - g.npml;
  double2 r = make_double2(0.0, 0.0);
  if (core) r = cscale(cmul(un[t], v[(size_t)(j - g.npml) * nxc + (i - g.npml)]), g.omega * g.omega);
  out[t] = r;
}

// out(c) = alpha v(c) + omega^2 sum_k conj(u_k) lambda_k (node of c) + gcoef gamma(node of c);
// real_only keeps the real part (the real-constrained step).  v may be NULL when alpha = 0.
__global__ void k_gather_PH(Grid g, int K, int nxc, double alpha, const double2 *__restrict__ v, double gcoef,
                            const double2 *__restrict__ un, const double2 *__restrict__ lam, int real_only,
                            double2 *__restrict__ out) {
  const int nzc = g.nz - 2 * g.npml;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)nxc * nzc) return;
  const size_t Nu = (size_t)g.nx * g.nz;
  const int ic = (int)(c % nxc), jc = (int)(c / nxc);
  const size_t p = (size_t)(jc + g.npml) * g.nx + ic + g.npml;
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < K; ++k) acc = cadd(acc, cmulc(un[(size_t)k * Nu + p], lam[(size_t)k * Nu + p]));
  double2 r = cscale(acc, g.omega * g.omega);
  if (v) r = cadd(r, cscale(v[c], alpha));
  r.x += gcoef * g.gamma[p];
  if (real_only) r.y = 0.0;
  out[c] = r;
}

__global__ void k_c128_to_c64(int64_t n, const double2 *__restrict__ x, float2 *y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < n; t += (int64_t)gridDim.x * blockDim.x) y[t] = make_float2((float)x[t].x, (float)x[t].y);
}
__global__ void k_c64_to_c128(int64_t n, const float2 *__restrict__ x, double2 *y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < n; t += (int64_t)gridDim.x * blockDim.x) y[t] = make_double2(x[t].x, x[t].y);
}

inline dim3 field_grid(const kf_problem *p, int zdim = 1) {
  return dim3((p->nx + BX - 1) / BX, (p->nz + BY - 1) / BY, zdim);
}
inline unsigned blocks_for(int64_t n, int bs = 256) {
  int64_t b = (n + bs - 1) / bs;
  return (unsigned)(b < 1 ? 1 : (b > 65535 * 16 ? 65535 * 16 : b));
}

}  // namespace

#define LAUNCH_CHECK()                                                              \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) {                                                         \
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_));     \
      return KF_EHIP;                                                               \
    }                                                                               \
  } while (0)

kf_status launch_pml(kf_problem *p, const kf_desc &d) {
  hipLaunchKernelGGL(k_stretch, dim3((p->nx + 256) / 256), dim3(256), 0, p->stream, p->nx, p->h, p->npml,
                     p->omega, d.pml_r0, d.pml_cref, p->xn, p->ixh);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_stretch, dim3((p->nz + 256) / 256), dim3(256), 0, p->stream, p->nz, p->h, p->npml,
                     p->omega, d.pml_r0, d.pml_cref, p->zn, p->izh);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_stretch(hipStream_t s, int n, double h, int npml, double omega, double r0, double cref, double2 *fn,
                         double2 *ifh) {
  hipLaunchKernelGGL(k_stretch, dim3((n + 256) / 256), dim3(256), 0, s, n, h, npml, omega, r0, cref, fn, ifh);
  LAUNCH_CHECK();
  return KF_OK;
}

template <typename R>
kf_status launch_stencil(kf_problem *p, int adjoint, const cplx<R> *x, cplx<R> *y) {
  ProfScope ps(p, PROF_STENCIL);
  const unsigned chunks = (unsigned)((p->Nu + KKT_WG - 1) / KKT_WG);
  const dim3 grid(chunks * (unsigned)((p->K + STEN_KPG - 1) / STEN_KPG));
  if (adjoint)
    hipLaunchKernelGGL((k_stencil<R, true>), grid, dim3(KKT_WG), 0, p->stream, p->grid(), p->K, chunks, x, y);
  else
    hipLaunchKernelGGL((k_stencil<R, false>), grid, dim3(KKT_WG), 0, p->stream, p->grid(), p->K, chunks, x, y);
  LAUNCH_CHECK();
  return KF_OK;
}
template kf_status launch_stencil<double>(kf_problem *, int, const double2 *, double2 *);
template kf_status launch_stencil<float>(kf_problem *, int, const float2 *, float2 *);

// y = M xi.  part / part_groups: buffer of the source groups' parts of the control
// row ([groups][Ng] c128) and the most groups it holds.
static kf_status launch_kkt_apply_into(kf_problem *p, const double2 *xi, double2 *y, double2 *part,
                                       int part_groups) {
  if (!p->kkt_resident) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_kkt_apply, KKT_WG, 0) != hipSuccess) {
      set_error("kkt_apply: device query failed");
      return KF_EHIP;
    }
    p->kkt_resident = ncu * (per > 0 ? per : 1);
  }
  // Source groups.  When the operands fit the 256 MB Infinity Cache, one round of
  // resident workgroups in lock step keeps the halo rows in L2.  When they stream from
  // HBM, many short workgroups (about 5 sources each) keep more loads in flight, which
  // pays for the larger per-group part of the control row.
  const unsigned chunks = (unsigned)((p->Nu + KKT_WG - 1) / KKT_WG);
  const double bytes = (double)p->Nu * (80.0 * p->K + 8.0);
  int groups = bytes <= 192e6 ? (int)(p->kkt_resident / chunks) : (p->K + 4) / 5;
  groups = groups < 1 ? 1 : (groups > part_groups ? part_groups : groups);
  const int kpg = (p->K + groups - 1) / groups;
  groups = (p->K + kpg - 1) / kpg;
  {
    // algorithmic bytes: du, lambda, u_n read and y_u, y_lambda written per node and
    // source; gamma per node; ds read and y_s written per control node
    ProfScope ps(p, PROF_KKT, bytes + 32.0 * (double)p->Ng);
    hipLaunchKernelGGL(k_kkt_apply, dim3(chunks * groups), dim3(KKT_WG), 0, p->stream, p->grid(), p->K, kpg,
                       p->nxc, chunks, p->eps, xi, p->u_n, y, part);
    LAUNCH_CHECK();
    if (groups > 1) {
      hipLaunchKernelGGL(k_kkt_ys_finish, dim3((unsigned)((p->Ng + 255) / 256)), dim3(256), 0, p->stream,
                         (size_t)p->Ng, groups, p->eps, p->omega * p->omega, xi + (size_t)p->K * p->Nu,
                         part, y + (size_t)p->K * p->Nu);
      LAUNCH_CHECK();
    }
  }
  int n = p->K * p->nru;
  hipLaunchKernelGGL(k_kkt_F, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->K, p->nru, p->d_rnode, p->d_wsq,
                     (size_t)p->Nu, xi, y);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_kkt_apply(kf_problem *p, const double2 *xi, double2 *y) {
  return launch_kkt_apply_into(p, xi, y, p->ys_part, p->kkt_groups_max);
}

// ---------------------------------------------------------------------------
// The KKT matvec for callers that cannot allocate (graph capture, serving loops):
// the source groups' parts of the control row go to a file-scope device array
// instead of the problem's own buffer.  Each GPU holds its copy of the array for the
// life of the process; its device address is looked up once per device.  Every part
// the finish kernel reads is written by the same launch first, so nothing needs
// clearing; calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;   // KF_NOALLOC_SCRATCH_BYTES
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];
static_assert(NOALLOC_SCRATCH_BYTES == KF_NOALLOC_SCRATCH_BYTES, "header and library agree on the scratch size");

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double2 *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static kf_status scratch_address(double2 **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) { set_error("device index out of range"); return KF_EHIP; }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
      return KF_EHIP;
    }
    scratch_ptr[dev] = (double2 *)ptr;
  }
  *out = scratch_ptr[dev];
  return KF_OK;
}

kf_status launch_kkt_apply_noalloc(kf_problem *p, const double2 *xi, double2 *y) {
  const size_t per_group = sizeof(double2) * (size_t)p->Ng;
  if (per_group > NOALLOC_SCRATCH_BYTES) {
    set_error("kkt_apply_noalloc: the control row (" + std::to_string(per_group) +
              " bytes) exceeds the scratch array (" + std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes)");
    return KF_ESHAPE;
  }
  double2 *part = nullptr;
  kf_status st = scratch_address(&part);
  if (st != KF_OK) return st;
  const size_t fit = NOALLOC_SCRATCH_BYTES / per_group;
  return launch_kkt_apply_into(p, xi, y, part, (int)std::min<size_t>(fit, (size_t)p->kkt_groups_max));
}

kf_status launch_precond_stage2(kf_problem *p, const double2 *y, double2 *z) {
  ProfScope ps(p, PROF_PRECOND);
  hipLaunchKernelGGL(k_precond_stage2, dim3((unsigned)((p->Nu + 63) / 64)), dim3(64, S2_G), 0, p->stream,
                     p->grid(), p->K, p->nxc, p->eps, y, p->u_n, z);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_sources(kf_problem *p, double2 *f) {
  int64_t n = (int64_t)p->K * p->Nu;
  hipLaunchKernelGGL(k_sources, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, p->K, (size_t)p->Nu,
                     p->d_src, 1.0 / (p->h * p->h), f);
  LAUNCH_CHECK();
  return KF_OK;
}

// residual buffers live in p->red_out-adjacent scratch owned by the caller (api.hip)
kf_status launch_residual(kf_problem *p, const double2 *d_obs, const double2 *u, double2 *r, double2 *wr) {
  int n = p->K * p->nrec;
  hipLaunchKernelGGL(k_residual, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->K, p->nrec, (size_t)p->Nu,
                     p->d_rec, p->d_w, d_obs, u, r, wr);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_rhs(kf_problem *p, const double2 *r, const int32_t *rptr, const int32_t *rlist, double2 *b,
                     int reg_on_update) {
  HIP_TRY(hipMemsetAsync(b, 0, sizeof(double2) * p->Nxi, p->stream));
  int n = p->K * p->nru;
  hipLaunchKernelGGL(k_rhs_u, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->K, p->nru, p->nrec,
                     (size_t)p->Nu, p->d_rnode, rptr, rlist, p->d_w, r, b);
  LAUNCH_CHECK();
  if (!reg_on_update) {
    int ng = (int)p->Ng;
    hipLaunchKernelGGL(k_rhs_s, dim3((ng + 255) / 256), dim3(256), 0, p->stream, p->nx, p->npml, p->nxc, p->nzc,
                       p->eps, p->gamma, b + (size_t)p->K * p->Nu);
    LAUNCH_CHECK();
  }
  return KF_OK;
}

kf_status launch_update_gamma(kf_problem *p, const double2 *ds, double *target) {
  int ng = (int)p->Ng;
  hipLaunchKernelGGL(k_update_gamma, dim3((ng + 255) / 256), dim3(256), 0, p->stream, p->nx, p->npml, p->nxc,
                     p->nzc, ds, target);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_grad_gamma(kf_problem *p, const void *u, const void *mu, int c64, double *grad) {
  if (c64)
    hipLaunchKernelGGL(k_grad_gamma<float2>, field_grid(p), dim3(BX, BY), 0, p->stream, p->grid(), p->K,
                       (const float2 *)u, (const float2 *)mu, grad);
  else
    hipLaunchKernelGGL(k_grad_gamma<double2>, field_grid(p), dim3(BX, BY), 0, p->stream, p->grid(), p->K,
                       (const double2 *)u, (const double2 *)mu, grad);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_axpy_field(kf_problem *p, int64_t n, double2 a, const double2 *x, double2 *y) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(256), 0, p->stream, n, a, x, y);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status launch_axpby_field(kf_problem *p, int64_t n, double2 a, const double2 *x, double2 b, double2 *y) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(256), 0, p->stream, n, a, x, b, y);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_scatter_P(kf_problem *p, const double2 *v, double2 *out) {
  const int64_t n = (int64_t)p->K * p->Nu;
  hipLaunchKernelGGL(k_scatter_P, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, p->grid(), p->K,
                     p->nxc, p->u_n, v, out);
  LAUNCH_CHECK();
  return KF_OK;
}

// out = Q^T W^2 Q x for every source (zero away from the receivers)
kf_status launch_apply_F(kf_problem *p, const double2 *x, double2 *out) {
  HIP_TRY(hipMemsetAsync(out, 0, sizeof(double2) * p->K * p->Nu, p->stream));
  int n = p->K * p->nru;
  hipLaunchKernelGGL(k_kkt_F, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->K, p->nru, p->d_rnode, p->d_wsq,
                     (size_t)p->Nu, x, out);
  LAUNCH_CHECK();
  return KF_OK;
}

// out = Q^T W^2 r for every source, r the data residual [K][nrec]
kf_status launch_rhs_u_field(kf_problem *p, const double2 *r, double2 *out) {
  HIP_TRY(hipMemsetAsync(out, 0, sizeof(double2) * p->K * p->Nu, p->stream));
  int n = p->K * p->nru;
  hipLaunchKernelGGL(k_rhs_u, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->K, p->nru, p->nrec,
                     (size_t)p->Nu, p->d_rnode, p->d_rptr, p->d_rlist, p->d_w, r, out);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_gather_PH(kf_problem *p, double alpha, const double2 *v, double gcoef, const double2 *lam,
                           int real_only, double2 *out) {
  hipLaunchKernelGGL(k_gather_PH, dim3((unsigned)((p->Ng + 255) / 256)), dim3(256), 0, p->stream, p->grid(), p->K,
                     p->nxc, alpha, v, gcoef, p->u_n, lam, real_only, out);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status launch_copy_c128_to_c64(kf_problem *p, int64_t n, const double2 *x, float2 *y) {
  hipLaunchKernelGGL(k_c128_to_c64, dim3(blocks_for(n)), dim3(256), 0, p->stream, n, x, y);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status launch_copy_c64_to_c128(kf_problem *p, int64_t n, const float2 *x, double2 *y) {
  hipLaunchKernelGGL(k_c64_to_c128, dim3(blocks_for(n)), dim3(256), 0, p->stream, n, x, y);
  LAUNCH_CHECK();
  return KF_OK;
}
