// Block-tridiagonal LU of the 5-point Helmholtz operator, swept over grid columns
// from both ends, and the batched forward / adjoint solves built on it.
//
// With unknowns grouped by grid column i (block size m = nz), A of Section 2 is
// block tridiagonal:  C_i x_{i-1} + D_i x_i + C_{i+1} x_{i+1} = b_i,
// D_i the (tridiagonal) column operator and C_i = diag(coupling of column i-1 and
// column i), the same in both directions because A is complex symmetric.
//
// Factorisation (FP64), meeting at column `mid`:
//   left   S_0 = D_0,            S_i = D_i - C_i T_{i-1} C_i,          i < mid
//   right  S_{n-1} = D_{n-1},    S_i = D_i - C_{i+1} T_{i+1} C_{i+1},  i > mid
//   middle S_mid = D_mid - C_mid T_{mid-1} C_mid - C_{mid+1} T_{mid+1} C_{mid+1}
//   T_i = S_i^-1 (dense Gauss-Jordan with partial pivoting), stored transposed.
// Solve: forward sweeps from both ends, the middle column, then back-substitution
// outward.  The adjoint uses A^H = conj(A):  A^H x = b  <=>  A conj(x) = conj(b).
//
// Every source shares the factors, so one factorisation per (gamma, omega) serves
// all K forward and adjoint block solves of the stacked system (Section 2) and
// every preconditioner application (Section 5).
#include "common.h"

namespace {

constexpr int FAC_THREADS = 1024;

// In-place Gauss-Jordan inversion of the row-major m x m matrix S (global memory),
// then writes the inverse transposed into Tt.  Called by a whole workgroup.
__device__ void gj_invert_store(double2 *S, int m, double2 *Tt, double2 *prow, double2 *fcol, int *piv,
                                double *red_v, int *red_i) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < m; ++k) {
    // pivot search: max |S[j][k]| over j >= k (ties -> smallest j)
    double best = -1.0; int bi = k;
    for (int j = k + tid; j < m; j += nt) {
      double a = cabs2(S[(size_t)j * m + k]);
      if (a > best) { best = a; bi = j; }
    }
    red_v[tid] = best; red_i[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        double a = red_v[tid + s]; int ai = red_i[tid + s];
        if (a > red_v[tid] || (a == red_v[tid] && ai < red_i[tid])) { red_v[tid] = a; red_i[tid] = ai; }
      }
      __syncthreads();
    }
    const int pr = red_i[0];
    if (tid == 0) piv[k] = pr;
    if (pr != k) {
      for (int l = tid; l < m; l += nt) {
        double2 a = S[(size_t)k * m + l];
        S[(size_t)k * m + l] = S[(size_t)pr * m + l];
        S[(size_t)pr * m + l] = a;
      }
    }
    __syncthreads();
    const double2 d = cdiv(make_double2(1.0, 0.0), S[(size_t)k * m + k]);
    for (int l = tid; l < m; l += nt) {
      double2 v = (l == k) ? d : cmul(S[(size_t)k * m + l], d);
      prow[l] = v;
      fcol[l] = (l == k) ? make_double2(0.0, 0.0) : S[(size_t)l * m + k];
    }
    __syncthreads();
    for (int l = tid; l < m; l += nt) S[(size_t)k * m + l] = prow[l];
    for (size_t e = tid; e < (size_t)m * m; e += nt) {
      int j = (int)(e / m), l = (int)(e % m);
      if (j == k) continue;
      double2 a = (l == k) ? make_double2(0.0, 0.0) : S[e];
      S[e] = csub(a, cmul(fcol[j], prow[l]));
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, in reverse order
  if (tid == 0) {
    for (int c = 0; c < m; ++c) red_i[c] = c;
    for (int k = m - 1; k >= 0; --k) {
      int a = red_i[k]; red_i[k] = red_i[piv[k]]; red_i[piv[k]] = a;
    }
  }
  __syncthreads();
  // Tt[c][j] = Sinv[j][c] = S[j][colsrc[c]]
  for (size_t e = tid; e < (size_t)m * m; e += nt) {
    int c = (int)(e / m), j = (int)(e % m);
    Tt[e] = S[(size_t)j * m + red_i[c]];
  }
  __syncthreads();
}

// S = D_i - C_a Tprev C_a (- C_b Tnext C_b), row-major.  ca/cb: column index whose
// coupling weights scale the correction, or -1 for none.
__device__ void build_schur(const Grid &g, int m, int i, const double2 *Tprev, int ca, const double2 *Tnext, int cb,
                            double2 *S) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (size_t e = tid; e < (size_t)m * m; e += nt) {
    int j = (int)(e / m), l = (int)(e % m);
    double2 v = make_double2(0.0, 0.0);
    if (ca >= 0) {  // Tprev[j][l] = Tt_prev[l][j]
      double2 t = Tprev[(size_t)l * m + j];
      v = csub(v, cmul(cmul(coupling_x(g, ca, j), t), coupling_x(g, ca, l)));
    }
    if (cb >= 0) {
      double2 t = Tnext[(size_t)l * m + j];
      v = csub(v, cmul(cmul(coupling_x(g, cb, j), t), coupling_x(g, cb, l)));
    }
    S[e] = v;
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) {
    Stencil5 s = stencil_at(g, i, j);
    size_t d = (size_t)j * m + j;
    S[d] = cadd(S[d], s.cc);
    if (j > 0) S[d - 1] = cadd(S[d - 1], s.czm);
    if (j + 1 < m) S[d + 1] = cadd(S[d + 1], s.czp);
  }
  __syncthreads();
}

// blockIdx.x = 0: left sweep over columns 0..mid-1; 1: right sweep over nx-1..mid+1.
// mode 1: the middle column (one block).
__global__ __launch_bounds__(FAC_THREADS) void k_blu_factor(Grid g, int mid, int mode, double2 *T, double2 *work) {
  extern __shared__ unsigned char smem[];
  const int m = g.nz;
  double2 *prow = (double2 *)smem;
  double2 *fcol = prow + m;
  int *piv = (int *)(fcol + m);
  double *red_v = (double *)(piv + ((m + 1) & ~1));
  int *red_i = (int *)(red_v + FAC_THREADS);
  const size_t mm = (size_t)m * m;
  double2 *S = work + (size_t)blockIdx.x * mm;
  if (mode == 0) {
    if (blockIdx.x == 0) {
      for (int i = 0; i < mid; ++i) {
        build_schur(g, m, i, i > 0 ? T + (size_t)(i - 1) * mm : nullptr, i > 0 ? i : -1, nullptr, -1, S);
        gj_invert_store(S, m, T + (size_t)i * mm, prow, fcol, piv, red_v, red_i);
      }
    } else {
      for (int i = g.nx - 1; i > mid; --i) {
        bool has = i + 1 < g.nx;
        build_schur(g, m, i, has ? T + (size_t)(i + 1) * mm : nullptr, has ? i + 1 : -1, nullptr, -1, S);
        gj_invert_store(S, m, T + (size_t)i * mm, prow, fcol, piv, red_v, red_i);
      }
    }
  } else {
    bool hl = mid > 0, hr = mid + 1 < g.nx;
    build_schur(g, m, mid, hl ? T + (size_t)(mid - 1) * mm : nullptr, hl ? mid : -1,
                hr ? T + (size_t)(mid + 1) * mm : nullptr, hr ? mid + 1 : -1, S);
    gj_invert_store(S, m, T + (size_t)mid * mm, prow, fcol, piv, red_v, red_i);
  }
}

template <typename R> __device__ inline cplx<R> to_r(double2 a) { return mk<R>((R)a.x, (R)a.y); }
template <typename R> __device__ inline cplx<R> to_r(float2 a) { return mk<R>((R)a.x, (R)a.y); }
template <typename IO> __device__ inline IO from_r(double2 a);
template <> __device__ inline double2 from_r<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_r<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <typename IO> __device__ inline IO from_r(float2 a);
template <> __device__ inline double2 from_r<double2>(float2 a) { return make_double2(a.x, a.y); }
template <> __device__ inline float2 from_r<float2>(float2 a) { return a; }

// Forward sweeps: side 0 computes y_i for i = 0..mid-1, side 1 for i = nx-1..mid+1.
// T: factors of type cplx<R> ([nx][m][m], transposed); b, x: IO type [K][nz][nx].
template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_fwd(Grid g, int K, int mid, const cplx<R> *__restrict__ T, const IO *b, IO *x) {
  using C = cplx<R>;
  extern __shared__ unsigned char smem[];
  const int m = g.nz;
  C *v = (C *)smem;          // [NS][m] previous y
  C *w = v + NS * m;         // [NS][m] right-hand side of this column
  const int tid = threadIdx.x, nt = blockDim.x;
  const int k0 = blockIdx.x * NS;
  const int side = blockIdx.y;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  int cnt = side == 0 ? mid : g.nx - 1 - mid;
  for (int step = 0; step < cnt; ++step) {
    const int i = side == 0 ? step : g.nx - 1 - step;
    const int cc = side == 0 ? i : i + 1;  // coupling column to the previous block
    for (int j = tid; j < m; j += nt) {
      C cj = step > 0 ? to_r<R>(coupling_x(g, cc, j)) : mk<R>(0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        int k = k0 + s;
        C r = mk<R>(0, 0);
        if (k < K) {
          r = to_r<R>(b[k * Nu + (size_t)j * g.nx + i]);
          if (ADJ) r = cconj(r);
          if (step > 0) r = csub(r, cmul(cj, v[s * m + j]));
        }
        w[s * m + j] = r;
      }
    }
    __syncthreads();
    const C *Ti = T + (size_t)i * mm;
    for (int j = tid; j < m; j += nt) {
      C acc[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
#pragma unroll 4
      for (int l = 0; l < m; ++l) {
        C t = Ti[(size_t)l * m + j];
#pragma unroll
        for (int s = 0; s < NS; ++s) cfma(acc[s], t, w[s * m + l]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        v[s * m + j] = acc[s];
        int k = k0 + s;
        if (k < K) x[k * Nu + (size_t)j * g.nx + i] = from_r<IO>(acc[s]);
      }
    }
    __syncthreads();
  }
}

// Middle column: x_mid = T_mid (b_mid - C_mid y_{mid-1} - C_{mid+1} y_{mid+1}).
template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_mid(Grid g, int K, int mid, const cplx<R> *__restrict__ T, const IO *b, IO *x,
                          cplx<R> *xmid) {
  using C = cplx<R>;
  extern __shared__ unsigned char smem[];
  const int m = g.nz;
  C *w = (C *)smem;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int k0 = blockIdx.x * NS;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  for (int j = tid; j < m; j += nt) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      int k = k0 + s;
      C r = mk<R>(0, 0);
      if (k < K) {
        const size_t base = k * Nu + (size_t)j * g.nx;
        r = to_r<R>(b[base + mid]);
        if (ADJ) r = cconj(r);
        if (mid > 0) r = csub(r, cmul(to_r<R>(coupling_x(g, mid, j)), to_r<R>(x[base + mid - 1])));
        if (mid + 1 < g.nx) r = csub(r, cmul(to_r<R>(coupling_x(g, mid + 1, j)), to_r<R>(x[base + mid + 1])));
      }
      w[s * m + j] = r;
    }
  }
  __syncthreads();
  const C *Ti = T + (size_t)mid * mm;
  for (int j = tid; j < m; j += nt) {
    C acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
#pragma unroll 4
    for (int l = 0; l < m; ++l) {
      C t = Ti[(size_t)l * m + j];
#pragma unroll
      for (int s = 0; s < NS; ++s) cfma(acc[s], t, w[s * m + l]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      int k = k0 + s;
      if (k < K) {
        xmid[(size_t)k * m + j] = acc[s];
        x[k * Nu + (size_t)j * g.nx + mid] = from_r<IO>(ADJ ? cconj(acc[s]) : acc[s]);
      }
    }
  }
}

// Back-substitution outward from the middle: side 0: x_i = y_i - T_i C_{i+1} x_{i+1}
// (i = mid-1..0); side 1: x_i = y_i - T_i C_i x_{i-1} (i = mid+1..nx-1).
template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_bwd(Grid g, int K, int mid, const cplx<R> *__restrict__ T, IO *x, const cplx<R> *xmid) {
  using C = cplx<R>;
  extern __shared__ unsigned char smem[];
  const int m = g.nz;
  C *w = (C *)smem;  // [NS][m] coupled previous x
  const int tid = threadIdx.x, nt = blockDim.x;
  const int k0 = blockIdx.x * NS;
  const int side = blockIdx.y;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  C xr[NS][4];  // rows owned by this thread (m <= 4 * blockDim.x)
  // start from x_mid
  for (int j = tid, q = 0; j < m; j += nt, ++q)
#pragma unroll
    for (int s = 0; s < NS; ++s) xr[s][q] = (k0 + s < K) ? xmid[(size_t)(k0 + s) * m + j] : mk<R>(0, 0);
  int cnt = side == 0 ? mid : g.nx - 1 - mid;
  for (int step = 0; step < cnt; ++step) {
    const int i = side == 0 ? mid - 1 - step : mid + 1 + step;
    const int cc = side == 0 ? i + 1 : i;
    for (int j = tid, q = 0; j < m; j += nt, ++q) {
      C cj = to_r<R>(coupling_x(g, cc, j));
#pragma unroll
      for (int s = 0; s < NS; ++s) w[s * m + j] = cmul(cj, xr[s][q]);
    }
    __syncthreads();
    const C *Ti = T + (size_t)i * mm;
    for (int j = tid, q = 0; j < m; j += nt, ++q) {
      C acc[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
#pragma unroll 4
      for (int l = 0; l < m; ++l) {
        C t = Ti[(size_t)l * m + j];
#pragma unroll
        for (int s = 0; s < NS; ++s) cfma(acc[s], t, w[s * m + l]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        int k = k0 + s;
        if (k < K) {
          size_t o = k * Nu + (size_t)j * g.nx + i;
          C y = to_r<R>(x[o]);
          C xi = csub(y, acc[s]);
          xr[s][q] = xi;
          x[o] = from_r<IO>(ADJ ? cconj(xi) : xi);
        }
      }
    }
    __syncthreads();
  }
}

inline int sweep_threads(int m) {
  int t = ((m + 63) / 64) * 64;
  return t > 512 ? 512 : (t < 64 ? 64 : t);
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

kf_status blu_factor(kf_problem *p, int which) {
  const int m = p->nz;
  const size_t mm = (size_t)m * m;
  if (which & 1) {
    if (!p->have_T64) {
      ProfScope ps(p, PROF_FACTOR);
      Grid g = p->grid();
      size_t smem = 2 * m * sizeof(double2) + ((m + 1) & ~1) * sizeof(int) + FAC_THREADS * (sizeof(double) + sizeof(int));
      hipLaunchKernelGGL(k_blu_factor, dim3(2), dim3(FAC_THREADS), smem, p->stream, g, p->mid, 0, p->T64, p->fac_work);
      LAUNCH_CHECK();
      hipLaunchKernelGGL(k_blu_factor, dim3(1), dim3(FAC_THREADS), smem, p->stream, g, p->mid, 1, p->T64, p->fac_work);
      LAUNCH_CHECK();
      p->have_T64 = true;
    }
  }
  if (which & 2) {
    if (!p->have_T64) {
      kf_status st = blu_factor(p, 1);
      if (st != KF_OK) return st;
    }
    if (!p->have_T32) {
      kf_status st = launch_copy_c128_to_c64(p, (int64_t)p->nx * mm, p->T64, p->T32);
      if (st != KF_OK) return st;
      p->have_T32 = true;
    }
  }
  return KF_OK;
}

namespace {
template <typename R, typename IO, bool ADJ>
kf_status sweep(kf_problem *p, const cplx<R> *T, const IO *rhs, IO *x, cplx<R> *xmid) {
  ProfScope ps(p, PROF_SWEEP);
  constexpr int NS = 1;
  const int m = p->nz;
  Grid g = p->grid();
  int groups = (p->K + NS - 1) / NS;
  int nt = sweep_threads(m);
  size_t smem = 2 * NS * m * sizeof(cplx<R>);
  hipLaunchKernelGGL((k_blu_fwd<R, IO, ADJ, NS>), dim3(groups, 2), dim3(nt), smem, p->stream, g, p->K, p->mid, T, rhs, x);
  LAUNCH_CHECK();
  hipLaunchKernelGGL((k_blu_mid<R, IO, ADJ, NS>), dim3(groups), dim3(nt), smem, p->stream, g, p->K, p->mid, T, rhs, x, xmid);
  LAUNCH_CHECK();
  hipLaunchKernelGGL((k_blu_bwd<R, IO, ADJ, NS>), dim3(groups, 2), dim3(nt), smem, p->stream, g, p->K, p->mid, T, x, xmid);
  LAUNCH_CHECK();
  return KF_OK;
}
}  // namespace

template <>
kf_status blu_solve<double>(kf_problem *p, int adjoint, const double2 *rhs, double2 *x) {
  kf_status st = blu_factor(p, 1);
  if (st != KF_OK) return st;
  return adjoint ? sweep<double, double2, true>(p, p->T64, rhs, x, p->xmid)
                 : sweep<double, double2, false>(p, p->T64, rhs, x, p->xmid);
}
template <>
kf_status blu_solve<float>(kf_problem *p, int adjoint, const float2 *rhs, float2 *x) {
  kf_status st = blu_factor(p, 2);
  if (st != KF_OK) return st;
  return adjoint ? sweep<float, float2, true>(p, p->T32, rhs, x, p->xmid32)
                 : sweep<float, float2, false>(p, p->T32, rhs, x, p->xmid32);
}
kf_status blu_solve_mixed_io(kf_problem *p, int adjoint, const double2 *rhs, double2 *x) {
  kf_status st = blu_factor(p, 2);
  if (st != KF_OK) return st;
  return adjoint ? sweep<float, double2, true>(p, p->T32, rhs, x, p->xmid32)
                 : sweep<float, double2, false>(p, p->T32, rhs, x, p->xmid32);
}
