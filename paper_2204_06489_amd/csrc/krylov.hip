// Krylov building blocks: deterministic wave64 reductions (fixed-order two-stage,
// no atomics), multi-dot / multi-axpy for classical Gram-Schmidt, and the small
// dense Hessenberg algebra of flexible GMRES kept on the device.
#include "common.h"

namespace {

constexpr int RB = 256;      // reduction block size (4 wavefronts)
constexpr int RG = 1024;     // reduction grid size (fixed => fixed summation order)
constexpr int MDOT = 16;     // vectors per multi-dot sweep (at most): 32 accumulators cost occupancy (4.0 vs 6.1 TB/s)
constexpr int FDOT = 8;      // dot products carried by the fused update-and-dot pass

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of NV doubles per thread; result valid in thread 0.  The values go
// through LDS eight at a time (lds: [8][RB] doubles, plus NV results), so that the
// compiler does not keep NV wave reductions in flight at once: the order of the sums
// is fixed, the register footprint small.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *lds /*[8 * RB + NV]*/) {
  double *res = lds + 8 * RB;
  const int tid = threadIdx.x;
#pragma unroll
  for (int c0 = 0; c0 < NV; c0 += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (c0 + k < NV) lds[k * RB + tid] = v[c0 + k];
    __syncthreads();
    // 8 rows of RB values: 32 lanes per row, each adds RB / 32 values, then a
    // 32-lane shuffle tree
    {
      const int k = tid >> 5, l = tid & 31;
      double s = 0.0;
      if (k < 8 && c0 + k < NV) {
#pragma unroll
        for (int i = 0; i < RB / 32; ++i) s += lds[k * RB + l + 32 * i];
      }
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
      if (k < 8 && l == 0 && c0 + k < NV) res[c0 + k] = s;
    }
    __syncthreads();
  }
  if (tid == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = res[q];
}

// partial[blockIdx][0..1] = sum conj(a) b over the block's grid-stride share
__global__ __launch_bounds__(RB) void k_dot_partial(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                    int64_t n, double *partial) {
  __shared__ double lds[8 * RB + 2];
  double v[2] = {0.0, 0.0};
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)RG * RB) {
    double2 x = a[t], y = b[t];
    v[0] += x.x * y.x + x.y * y.y;
    v[1] += x.x * y.y - x.y * y.x;
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) { partial[2 * blockIdx.x] = v[0]; partial[2 * blockIdx.x + 1] = v[1]; }
}

__global__ __launch_bounds__(RB) void k_norm2_partial(const double2 *__restrict__ a, int64_t n, double *partial,
                                                      const int *active) {
  if (active && *active == 0) return;
  __shared__ double lds[8 * RB + 1];
  double v[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)RG * RB) {
    double2 x = a[t];
    v[0] += x.x * x.x + x.y * x.y;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// sum the RG partials of nq quantities in fixed order; out[q] = sum (or sqrt for norms).
// One workgroup per quantity (grid-strided), so the order of each sum is fixed.
__global__ __launch_bounds__(RB) void k_finish(const double *__restrict__ partial, int nq, int stride, int take_sqrt,
                                               double *out, const int *active) {
  if (active && *active == 0) return;
  __shared__ double lds[8 * RB + 1];
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < RG; b += RB) v[0] += partial[(size_t)b * stride + q];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[q] = take_sqrt ? sqrt(v[0]) : v[0];
    __syncthreads();
  }
}

// number of non-finite entries (NaN or +-inf) of a real array: partial counts per block
__global__ __launch_bounds__(RB) void k_nonfinite_partial(const double *__restrict__ a, int64_t n, double *partial) {
  __shared__ double lds[8 * RB + 1];
  double v[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)RG * RB)
    if (!isfinite(a[t])) v[0] += 1.0;
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// h[q] = V_q^H w for q in [q0, q0 + NQ): partial sums per block; with `norm` also
// |w|^2 from the same sweep, stored after the 2 nv dot-product entries of the row.
// FIRST marks the first Gram-Schmidt pass's launches (always real work) apart from the
// second pass's (which return at once unless the step needs them), so that kernel
// traces time the two separately.
template <int NQ, bool FIRST>
__global__ __launch_bounds__(RB) void k_multidot_partial(const double2 *__restrict__ V, int q0, int nv,
                                                         const double2 *__restrict__ w, int64_t n, double *partial,
                                                         int stride, int norm, const int *active) {
  if (active && *active == 0) return;
  __shared__ double lds[8 * RB + 2 * NQ + 1];
  double v[2 * NQ + 1];
#pragma unroll
  for (int q = 0; q < 2 * NQ + 1; ++q) v[q] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)RG * RB) {
    double2 y = w[t];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q0 + q < nv) {
        double2 x = V[(size_t)(q0 + q) * n + t];
        v[2 * q] += x.x * y.x + x.y * y.y;
        v[2 * q + 1] += x.x * y.y - x.y * y.x;
      }
    }
    v[2 * NQ] += y.x * y.x + y.y * y.y;
  }
  block_sum<2 * NQ + 1>(v, lds);
  if (threadIdx.x == 0) {
    for (int q = 0; q < 2 * NQ; ++q)
      if (q0 + q / 2 < nv) partial[(size_t)blockIdx.x * stride + 2 * q0 + q] = v[q];
    if (norm) partial[(size_t)blockIdx.x * stride + 2 * nv] = v[2 * NQ];
  }
}

// One sweep of the multi-dot over vectors [q0, q0 + nq), nq <= MDOT, with the smaller
// template that holds them (8 or 16 vectors per sweep).
template <bool FIRST>
inline void launch_multidot(hipStream_t s, const double2 *V, int q0, int nq, int nv, const double2 *w, int64_t n,
                            double *partial, int stride, int norm, const int *active) {
  if (nq <= 8)
    hipLaunchKernelGGL((k_multidot_partial<8, FIRST>), dim3(RG), dim3(RB), 0, s, V, q0, nv, w, n, partial, stride,
                       norm, active);
  else
    hipLaunchKernelGGL((k_multidot_partial<16, FIRST>), dim3(RG), dim3(RB), 0, s, V, q0, nv, w, n, partial, stride,
                       norm, active);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));   // 16-byte access for the non-temporal builtins

// Fused Gram-Schmidt update: w <- (w - sum_{q<nv} V_q h_q) * scale[0] (scale NULL: 1),
// written back, while the same sweep accumulates the dot products V_q^H w (new w) for
// q < min(nv, FDOT) (WANT_DOTS) and |w|^2 (new w).  partial row of a block:
// [2 * FDOT dots | norm^2].
template <bool WANT_DOTS>
__global__ __launch_bounds__(RB) void k_axpy_dot_partial(const double2 *__restrict__ V, int nv,
                                                         const double2 *__restrict__ h, double2 *w, int64_t n,
                                                         double *partial, const double *scale, const int *active) {
  if (active && *active == 0) return;
  const double sc = scale ? scale[0] : 1.0;
  constexpr int NQ = WANT_DOTS ? FDOT : 0;
  __shared__ double lds[8 * RB + 2 * FDOT + 1];
  // h is read with uniform indices (scalar loads): the coefficients sit in SGPRs
  const double2 *__restrict__ hs = h;
  double v[2 * NQ + 1];
#pragma unroll
  for (int q = 0; q < 2 * NQ + 1; ++q) v[q] = 0.0;
  const int nd = nv < NQ ? nv : NQ;
#pragma unroll 1
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)RG * RB) {
    double2 y = w[t];
    double2 x[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      x[q] = q < nd ? V[(size_t)q * n + t] : make_double2(0.0, 0.0);
      if (q < nd) y = csub(y, cmul(x[q], hs[q]));   // h holds nv entries only
    }
    // the remaining vectors eight at a time, their loads in flight together (the
    // subtractions keep the ascending order); they and the new w are streamed once per
    // sweep, so they bypass the caches (non-temporal: 2% faster than cached accesses)
#pragma unroll 1
    for (int q0 = NQ; q0 < nv; q0 += 8) {
      double2 xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const dvec2 l = q0 + u < nv ? __builtin_nontemporal_load((const dvec2 *)&V[(size_t)(q0 + u) * n + t])
                                    : dvec2{0.0, 0.0};
        xv[u] = make_double2(l.x, l.y);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < nv) y = csub(y, cmul(xv[u], hs[q0 + u]));
    }
    y = cscale(y, sc);
    __builtin_nontemporal_store(dvec2{y.x, y.y}, (dvec2 *)&w[t]);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      v[2 * q] += x[q].x * y.x + x[q].y * y.y;
      v[2 * q + 1] += x[q].x * y.y - x[q].y * y.x;
    }
    v[2 * NQ] += y.x * y.x + y.y * y.y;
  }
  block_sum<2 * NQ + 1>(v, (double *)lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < 2 * NQ + 1; ++q) partial[(size_t)blockIdx.x * (2 * FDOT + 1) + q] = v[q];
}

// w += sign * sum_q V_q h_q
__global__ __launch_bounds__(RB) void k_multiaxpy(const double2 *__restrict__ V, int nv, const double2 *__restrict__ h,
                                                  double sign, double2 *w, int64_t n, const int *active) {
  if (active && *active == 0) return;
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)gridDim.x * RB) {
    double2 acc = w[t];
#pragma unroll 1
    for (int q0 = 0; q0 < nv; q0 += 8) {   // eight loads in flight, ascending order kept
      double2 xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = q0 + u < nv ? V[(size_t)(q0 + u) * n + t] : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < nv) {
          double2 hq = h[q0 + u];
          hq.x *= sign; hq.y *= sign;
          cfma(acc, xv[u], hq);
        }
    }
    w[t] = acc;
  }
}

// Gram-Schmidt decision before the update w' = w - V h (V orthonormal, so
// |w'|^2 = |w|^2 - |h|^2 up to rounding), from |w|^2 of the dot-product sweep:
//   |w'| >= max(eta, 0.1) |w|: the cancellation is mild, |w'| is taken from that
//     difference (relative error ~ nv eps |w|^2 / |w'|^2 <= 1e-13) and the update
//     writes the normalised vector w' / |w'| directly: flags (0, 0);
//   |w'| < eta |w| (test of Daniel, Gragg, Kaufman and Stewart): a second pass,
//     flags (1, 1);
//   otherwise (eta < 0.1 and strong cancellation): one pass, but |w'| is measured by
//     the update's sweep and a scaling pass follows: flags (0, 1).
// flags[0] asks for the second pass, flags[1] for the measured norm and the scaling;
// h2 is zeroed unless flags[0].  nrm[0] receives |w'| in the first case, scale[0] the
// factor the update applies (1 / |w'| or 1).
__global__ void k_gs_decide(int nv, const double2 *h1, const double *wn2, double eta, double2 *h2, int *flags,
                            double *nrm, double *scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nv; ++i) s += cabs2(h1[i]);
  const double w2 = wn2[0], nu2 = w2 - s;
  const double thr = eta > 0.1 ? eta : 0.1;
  int reorth = 0, measure = 0;
  if (nu2 >= thr * thr * w2 && nu2 > 0.0) {
    nrm[0] = sqrt(nu2);
    scale[0] = 1.0 / nrm[0];
  } else {
    reorth = (eta > 0.0 && !(nu2 >= eta * eta * w2)) ? 1 : 0;
    measure = 1;
    scale[0] = 1.0;
  }
  flags[0] = reorth;
  flags[1] = measure;
  if (!reorth)
    for (int i = 0; i < nv; ++i) h2[i] = make_double2(0.0, 0.0);
}

// per-source ||x_k||^2 partials: grid (RG/8, K)
__global__ __launch_bounds__(RB) void k_src_norm_partial(const double2 *__restrict__ x, int64_t n_per, double *partial) {
  __shared__ double lds[8 * RB + 1];
  const int k = blockIdx.y;
  const int nb = gridDim.x;
  double v[1] = {0.0};
  const double2 *xk = x + (size_t)k * n_per;
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n_per; t += (int64_t)nb * RB) {
    double2 a = xk[t];
    v[0] += a.x * a.x + a.y * a.y;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[(size_t)k * nb + blockIdx.x] = v[0];
}
__global__ void k_src_norm_finish(const double *__restrict__ partial, int nb, int K, double *out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(size_t)k * nb + b];
  out[k] = sqrt(s);
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

// p->red must hold RG * 2 * (max vectors) doubles
kf_status dot_c128(kf_problem *p, const double2 *a, const double2 *b, int64_t n, double2 *out_dev) {
  ProfScope ps(p, PROF_REDUCE);
  hipLaunchKernelGGL(k_dot_partial, dim3(RG), dim3(RB), 0, p->stream, a, b, n, p->red);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_finish, dim3(2), dim3(RB), 0, p->stream, p->red, 2, 2, 0, (double *)out_dev, nullptr);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status norm_c128(kf_problem *p, const double2 *a, int64_t n, double *out_dev, const int *active) {
  ProfScope ps(p, PROF_REDUCE);
  hipLaunchKernelGGL(k_norm2_partial, dim3(RG), dim3(RB), 0, p->stream, a, n, p->red, active);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, p->stream, p->red, 1, 1, 1, out_dev, active);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status count_nonfinite(kf_problem *p, const double *a, int64_t n, int64_t *count_host) {
  hipLaunchKernelGGL(k_nonfinite_partial, dim3(RG), dim3(RB), 0, p->stream, a, n, p->red);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, p->stream, p->red, 1, 1, 0, p->red_out, nullptr);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(p->host_pinned, p->red_out, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *count_host = (int64_t)p->host_pinned[0];
  return KF_OK;
}

kf_status multidot_c128(kf_problem *p, const double2 *V, int nv, const double2 *w, int64_t n, double2 *h_dev,
                        const int *active, double *nrm2_out) {
  // algorithmic bytes: the nv basis vectors and w read once
  ProfScope ps(p, nrm2_out ? PROF_GS_DOT : PROF_ORTH, 16.0 * (double)n * (nv + 1));
  const int stride = 2 * nv + 1;
  for (int q0 = 0; q0 < nv; q0 += MDOT) {
    if (nrm2_out)
      launch_multidot<true>(p->stream, V, q0, std::min(MDOT, nv - q0), nv, w, n, p->red, stride, q0 == 0, active);
    else
      launch_multidot<false>(p->stream, V, q0, std::min(MDOT, nv - q0), nv, w, n, p->red, stride, 0, active);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_finish, dim3(2 * nv), dim3(RB), 0, p->stream, p->red, 2 * nv, stride, 0, (double *)h_dev, active);
  LAUNCH_CHECK();
  if (nrm2_out) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, p->stream, p->red + 2 * nv, 1, stride, 0, nrm2_out, active);
    LAUNCH_CHECK();
  }
  return KF_OK;
}

kf_status multiaxpy_c128(kf_problem *p, const double2 *V, int nv, const double2 *h_dev, double sign, double2 *w,
                         int64_t n, const int *active) {
  ProfScope ps(p, PROF_ORTH);
  int64_t b = (n + RB - 1) / RB;
  unsigned grid = (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
  hipLaunchKernelGGL(k_multiaxpy, dim3(grid), dim3(RB), 0, p->stream, V, nv, h_dev, sign, w, n, active);
  LAUNCH_CHECK();
  return KF_OK;
}

// w <- w - V h (nv vectors); then |w| and, with h_out, the first min(nv, FDOT) entries
// of V^H w from the same sweep (the rest: multidot_rest_c128)
kf_status axpy_dot_c128(kf_problem *p, const double2 *V, int nv, const double2 *h, double2 *w, int64_t n,
                        double2 *h_out, double *nrm_out, const int *active, const double *scale,
                        const int *active_dots) {
  // algorithmic bytes: the nv basis vectors and w read, w written
  ProfScope ps(p, scale ? PROF_GS_UPDATE : PROF_ORTH, 16.0 * (double)n * (nv + 2));
  if (nv > 256) { set_error("too many Krylov vectors for the fused update"); return KF_EINVAL; }
  const int stride = 2 * FDOT + 1;
  const int *gate = scale ? nullptr : active;   // with a scale the update itself always runs
  if (h_out)
    hipLaunchKernelGGL(k_axpy_dot_partial<true>, dim3(RG), dim3(RB), 0, p->stream, V, nv, h, w, n, p->red, scale, gate);
  else
    hipLaunchKernelGGL(k_axpy_dot_partial<false>, dim3(RG), dim3(RB), 0, p->stream, V, nv, h, w, n, p->red, scale, gate);
  LAUNCH_CHECK();
  // norm: the last entry of each partial row
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, p->stream, p->red + (h_out ? 2 * FDOT : 0), 1, stride, 1, nrm_out,
                     active);
  LAUNCH_CHECK();
  if (h_out) {
    const int nd = nv < FDOT ? nv : FDOT;
    hipLaunchKernelGGL(k_finish, dim3(2 * nd), dim3(RB), 0, p->stream, p->red, 2 * nd, stride, 0, (double *)h_out,
                       active_dots ? active_dots : active);
    LAUNCH_CHECK();
  }
  return KF_OK;
}

kf_status gs_decide(kf_problem *p, int nv, const double2 *h1, const double *wn2, double eta, double2 *h2, int *flags,
                    double *nrm, double *scale) {
  ProfScope ps(p, PROF_ORTH);
  hipLaunchKernelGGL(k_gs_decide, dim3(1), dim3(64), 0, p->stream, nv, h1, wn2, eta, h2, flags, nrm, scale);
  LAUNCH_CHECK();
  return KF_OK;
}

// h_out[q] = V_q^H w for FDOT <= q < nv (the entries the fused sweep does not carry)
kf_status multidot_rest_c128(kf_problem *p, const double2 *V, int nv, const double2 *w, int64_t n, double2 *h_out,
                             const int *active) {
  ProfScope ps(p, PROF_ORTH);
  if (nv <= FDOT) return KF_OK;
  double *red2 = p->red + (size_t)RG * (2 * FDOT + 1);
  const int stride2 = 2 * nv;
  for (int q0 = FDOT; q0 < nv; q0 += MDOT) {
    launch_multidot<false>(p->stream, V, q0, std::min(MDOT, nv - q0), nv, w, n, red2, stride2, 0, active);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_finish, dim3(2 * (nv - FDOT)), dim3(RB), 0, p->stream, red2 + 2 * FDOT, 2 * (nv - FDOT), stride2,
                     0, (double *)(h_out + FDOT), active);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status per_source_norms(kf_problem *p, const double2 *x, int64_t n_per, int K, double *out_host) {
  ProfScope ps(p, PROF_REDUCE);
  const int nb = 64;
  hipLaunchKernelGGL(k_src_norm_partial, dim3(nb, K), dim3(RB), 0, p->stream, x, n_per, p->red);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_src_norm_finish, dim3((K + 63) / 64), dim3(64), 0, p->stream, p->red, nb, K, p->red_out);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(out_host, p->red_out, sizeof(double) * K, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return KF_OK;
}

namespace {

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes, previous
// Givens rotations applied, a new rotation annihilating H[j+1][j], and the
// least-squares right-hand side g updated; resid = |g[j+1]| is the GMRES
// residual norm estimate.  H is (m+1) x m column-major.
__global__ void k_arnoldi_finish(int j, int m, const double2 *h1, const double2 *h2, const double *nrm, double2 *H,
                                 double2 *cs, double2 *sn, double2 *g, double *resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double2 *col = H + (size_t)j * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = cadd(h1[i], h2 ? h2[i] : make_double2(0.0, 0.0));
  col[j + 1] = make_double2(nrm[0], 0.0);
  for (int i = 0; i < j; ++i) {
    double2 a = col[i], b = col[i + 1];
    double c = cs[i].x;
    double2 s = sn[i];
    col[i] = cadd(cscale(a, c), cmul(s, b));
    col[i + 1] = csub(cscale(b, c), cmulc(s, a));
  }
  double2 a = col[j], b = col[j + 1];
  double na = sqrt(cabs2(a)), nb = sqrt(cabs2(b));
  double r = sqrt(na * na + nb * nb);
  double c;
  double2 s;
  if (r == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); }
  else if (na == 0.0) { c = 0.0; s = make_double2(1.0, 0.0); }
  else {
    c = na / r;
    double2 ph = cscale(a, 1.0 / na);          // a / |a|
    s = cscale(cmul(ph, cconj(b)), 1.0 / r);   // (a/|a|) conj(b) / r
  }
  cs[j] = make_double2(c, 0.0);
  sn[j] = s;
  col[j] = cadd(cscale(a, c), cmul(s, b));
  col[j + 1] = make_double2(0.0, 0.0);
  double2 gj = g[j];
  g[j] = cscale(gj, c);
  g[j + 1] = csub(make_double2(0.0, 0.0), cmulc(s, gj));
  resid[0] = sqrt(cabs2(g[j + 1]));
}

__global__ void k_backsolve(int nj, int m, const double2 *H, const double2 *g, double2 *y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = nj - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int l = i + 1; l < nj; ++l) acc = csub(acc, cmul(H[(size_t)l * (m + 1) + i], y[l]));
    y[i] = cdiv(acc, H[(size_t)i * (m + 1) + i]);
  }
}

__global__ void k_set_g0(int m, const double *beta, double2 *g) {
  int t = threadIdx.x;
  for (int i = t; i <= m; i += blockDim.x) g[i] = make_double2(i == 0 ? beta[0] : 0.0, 0.0);
}

__global__ void k_scale_inv(int64_t n, const double *nrm, const double2 *x, double2 *y, const int *active) {
  if (active && *active == 0) return;
  double s = nrm[0] > 0.0 ? 1.0 / nrm[0] : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    y[t] = cscale(x[t], s);
}

__global__ void k_imag(int64_t n, const double2 *x, double2 *y) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    y[t] = make_double2(0.0, x[t].y);
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

kf_status arnoldi_finish(kf_problem *p, int j, int m, const double2 *h1, const double2 *h2, const double *nrm,
                         double2 *H, double2 *cs, double2 *sn, double2 *g, double *resid) {
  ProfScope ps(p, PROF_ORTH);
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, p->stream, j, m, h1, h2, nrm, H, cs, sn, g, resid);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status hess_backsolve(kf_problem *p, int nj, int m, const double2 *H, const double2 *g, double2 *y) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, p->stream, nj, m, H, g, y);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status set_g0(kf_problem *p, int m, const double *beta, double2 *g) {
  hipLaunchKernelGGL(k_set_g0, dim3(1), dim3(256), 0, p->stream, m, beta, g);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status scale_inv(kf_problem *p, int64_t n, const double *nrm, const double2 *x, double2 *y, const int *active) {
  ProfScope ps(p, PROF_ORTH);
  hipLaunchKernelGGL(k_scale_inv, dim3(grid_for(n)), dim3(256), 0, p->stream, n, nrm, x, y, active);
  LAUNCH_CHECK();
  return KF_OK;
}
kf_status imag_part(kf_problem *p, int64_t n, const double2 *x, double2 *y) {
  hipLaunchKernelGGL(k_imag, dim3(grid_for(n)), dim3(256), 0, p->stream, n, x, y);
  LAUNCH_CHECK();
  return KF_OK;
}
