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

// In-place Gauss-Jordan inversion of the row-major m x m matrix S (global memory),
// blocked by NB-column panels, then the inverse written transposed into Tt.  Called
// by a whole workgroup.
//
// For each panel the classical in-place Gauss-Jordan steps (partial pivoting over
// all rows, pivot row scaled, pivot column eliminated from every other row, the
// eliminated column replaced by the accumulated transform) run on the m x NB panel
// in LDS.  Their combined effect on every other column x is
//     x  <-  (P x with the panel's pivot rows zeroed) + Pan (P x)[pivot rows],
// P the panel's row interchanges and Pan the finished panel, which is one rank-NB
// update of the matrix (register tiles of TR x TC entries per thread).  After the
// last panel the row interchanges are undone as column interchanges.
constexpr int TR = 4, TC = 4;   // update tile per thread
constexpr int NB_MAX = 16;

// orders the LDS accesses of the lanes of one wavefront (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NB, int RMAX>
__device__ __forceinline__ void gj_invert_store(double2 *S, int m, double2 *Tt, double2 *pan /*[m][NB]*/,
                                                double2 *x1 /*[NB][m]*/, double2 *rowbuf /*[2][NB]*/, int *piv,
                                                int *perm /*[m]*/, double2 *tmp /*[NB][m] global*/) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int K0 = 0; K0 < m; K0 += NB) {
    const int nb = min(NB, m - K0);
    for (int r = tid; r < m; r += nt) perm[r] = r;
    __syncthreads();
    // Gauss-Jordan on the panel by wavefront 0, the panel held in registers: lane l
    // owns rows l, l + 64, ...  A pivot step is a shuffle reduction for the pivot, a
    // two-row exchange through LDS and register arithmetic; no workgroup barrier.
    if (wave == 0) {
      double2 v[RMAX][NB];
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int r = lane + 64 * t;
#pragma unroll
        for (int c = 0; c < NB; ++c) v[t][c] = (r < m && c < nb) ? S[(size_t)r * m + K0 + c] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (q < nb) {
          const int k = K0 + q;
          double best = -1.0;
          int bi = m;
#pragma unroll
          for (int t = 0; t < RMAX; ++t) {
            const int r = lane + 64 * t;
            if (r >= k && r < m) {
              double a = cabs2(v[t][q]);
              if (a > best) { best = a; bi = r; }
            }
          }
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            double ob = __shfl_xor(best, o, 64);
            int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
          }
          const int pr = bi;
          // rows k and pr to LDS (pr first)
#pragma unroll
          for (int t = 0; t < RMAX; ++t) {
            const int r = lane + 64 * t;
            if (r == pr)
#pragma unroll
              for (int c = 0; c < NB; ++c) rowbuf[c] = v[t][c];
            if (r == k)
#pragma unroll
              for (int c = 0; c < NB; ++c) rowbuf[NB + c] = v[t][c];
          }
          if (lane == 0) {
            piv[k] = pr;
            int a = perm[k]; perm[k] = perm[pr]; perm[pr] = a;
          }
          wave_sync();
          double2 prow[NB];
#pragma unroll
          for (int c = 0; c < NB; ++c) prow[c] = rowbuf[c];
          // the new row k is the old row pr, scaled; the pivot entry becomes 1 / pivot
          const double2 d = cdiv(make_double2(1.0, 0.0), prow[q]);
#pragma unroll
          for (int c = 0; c < NB; ++c) prow[c] = (c == q) ? d : cmul(prow[c], d);
#pragma unroll
          for (int t = 0; t < RMAX; ++t) {
            const int r = lane + 64 * t;
            if (r == k) {
#pragma unroll
              for (int c = 0; c < NB; ++c) v[t][c] = prow[c];
            } else {
              if (r == pr)   // the old row k moves to pr, then is eliminated like every other row
#pragma unroll
                for (int c = 0; c < NB; ++c) v[t][c] = rowbuf[NB + c];
              const double2 f = v[t][q];
#pragma unroll
              for (int c = 0; c < NB; ++c)
                v[t][c] = csub(c == q ? make_double2(0.0, 0.0) : v[t][c], cmul(f, prow[c]));
            }
          }
          wave_sync();   // rowbuf is rewritten by the next pivot step
        }
      }
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int r = lane + 64 * t;
        if (r < m)
#pragma unroll
          for (int c = 0; c < NB; ++c) pan[r * NB + c] = v[t][c];
      }
    }
    __syncthreads();
    // The panel's row interchanges on the other columns, as one permutation: the new
    // pivot-block rows go to x1, the old pivot-block rows are staged in tmp, and every
    // row outside the block that took part in an interchange receives the old
    // pivot-block row the interchanges moved there (perm[r] is its origin).
    for (int e = tid; e < nb * m; e += nt) {
      const int q = e / m, c = e % m;
      x1[e] = S[(size_t)perm[K0 + q] * m + c];
      tmp[e] = S[(size_t)(K0 + q) * m + c];
    }
    __syncthreads();
    for (int e = tid; e < nb * m; e += nt) {
      const int q = e / m, c = e % m;
      const int r = piv[K0 + q];
      if (r >= K0 + nb && perm[r] != r && !(c >= K0 && c < K0 + nb)) S[(size_t)r * m + c] = tmp[(size_t)(perm[r] - K0) * m + c];
    }
    __syncthreads();
    // rank-nb update of every column outside the panel (register tiles TR x TC)
    const int ntr = (m + TR - 1) / TR, ntc = (m + TC - 1) / TC;
    for (int t = tid; t < ntr * ntc; t += nt) {
      const int r0 = (t / ntc) * TR, c0 = (t % ntc) * TC;
      double2 acc[TR][TC];
#pragma unroll
      for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b) {
          int r = r0 + a, c = c0 + b;
          bool in = r < m && c < m && !(r >= K0 && r < K0 + nb) && !(c >= K0 && c < K0 + nb);
          acc[a][b] = in ? S[(size_t)r * m + c] : make_double2(0.0, 0.0);
        }
      for (int q = 0; q < nb; ++q) {
        double2 pr[TR], xc[TC];
#pragma unroll
        for (int a = 0; a < TR; ++a) pr[a] = (r0 + a < m) ? pan[(r0 + a) * NB + q] : make_double2(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < TC; ++b) xc[b] = (c0 + b < m) ? x1[q * m + c0 + b] : make_double2(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < TR; ++a)
#pragma unroll
          for (int b = 0; b < TC; ++b) cfma(acc[a][b], pr[a], xc[b]);
      }
#pragma unroll
      for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b) {
          int r = r0 + a, c = c0 + b;
          if (r < m && c < m && !(c >= K0 && c < K0 + nb)) S[(size_t)r * m + c] = acc[a][b];
        }
    }
    for (int e = tid; e < m * nb; e += nt) {
      int r = e / nb, q = e % nb;
      S[(size_t)r * m + K0 + q] = pan[r * NB + q];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, in reverse order
  if (tid == 0) {
    for (int c = 0; c < m; ++c) perm[c] = c;
    for (int k = m - 1; k >= 0; --k) {
      int a = perm[k]; perm[k] = perm[piv[k]]; perm[piv[k]] = a;
    }
  }
  __syncthreads();
  // Tt[c][j] = Sinv[j][c] = S[j][colsrc[c]]
  for (size_t e = tid; e < (size_t)m * m; e += nt) {
    int c = (int)(e / m), j = (int)(e % m);
    Tt[e] = S[(size_t)j * m + perm[c]];
  }
  __syncthreads();
}

// S = D_i - C_a Tprev C_a (- C_b Tnext C_b), row-major.  ca/cb: column index whose
// coupling weights scale the correction, or -1 for none.  cw: LDS scratch [2][m].
__device__ __forceinline__ void build_schur(const Grid &g, int m, int i, const double2 *Tprev, int ca, const double2 *Tnext, int cb,
                            double2 *S, double2 *cw) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < m; j += nt) {
    cw[j] = ca >= 0 ? coupling_x(g, ca, j) : make_double2(0.0, 0.0);
    cw[m + j] = cb >= 0 ? coupling_x(g, cb, j) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (size_t e = tid; e < (size_t)m * m; e += nt) {
    int j = (int)(e / m), l = (int)(e % m);
    double2 v = make_double2(0.0, 0.0);
    if (ca >= 0) v = csub(v, cmul(cmul(cw[j], Tprev[(size_t)l * m + j]), cw[l]));   // Tprev[j][l] = Tt[l][j]
    if (cb >= 0) v = csub(v, cmul(cmul(cw[m + j], Tnext[(size_t)l * m + j]), cw[m + l]));
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
// mode 1: the middle column (one block).  work: per block an m x m matrix and an
// NB x m staging area.
template <int NB, int RMAX>
__device__ __forceinline__ void blu_factor_body(const Grid &g, int mid, int mode, int side, double2 *T, double2 *work,
                                                unsigned char *smem) {
  const int m = g.nz;
  double2 *pan = (double2 *)smem;          // [m][NB]
  double2 *x1 = pan + (size_t)m * NB;      // [NB][m]
  double2 *cw = x1 + (size_t)m * NB;       // [2][m]
  double2 *prow = cw + 2 * (size_t)m;      // [2][NB] row exchange buffer
  int *piv = (int *)(prow + 2 * NB);       // [m]
  int *perm = piv + m;                     // [m]
  const size_t mm = (size_t)m * m;
  double2 *S = work + (size_t)side * (mm + (size_t)NB_MAX * m);
  double2 *tmp = S + mm;
  if (mode == 0) {
    if (side == 0) {
      for (int i = 0; i < mid; ++i) {
        build_schur(g, m, i, i > 0 ? T + (size_t)(i - 1) * mm : nullptr, i > 0 ? i : -1, nullptr, -1, S, cw);
        gj_invert_store<NB, RMAX>(S, m, T + (size_t)i * mm, pan, x1, prow, piv, perm, tmp);
      }
    } else {
      for (int i = g.nx - 1; i > mid; --i) {
        bool has = i + 1 < g.nx;
        build_schur(g, m, i, has ? T + (size_t)(i + 1) * mm : nullptr, has ? i + 1 : -1, nullptr, -1, S, cw);
        gj_invert_store<NB, RMAX>(S, m, T + (size_t)i * mm, pan, x1, prow, piv, perm, tmp);
      }
    }
  } else {
    bool hl = mid > 0, hr = mid + 1 < g.nx;
    build_schur(g, m, mid, hl ? T + (size_t)(mid - 1) * mm : nullptr, hl ? mid : -1,
                hr ? T + (size_t)(mid + 1) * mm : nullptr, hr ? mid + 1 : -1, S, cw);
    gj_invert_store<NB, RMAX>(S, m, T + (size_t)mid * mm, pan, x1, prow, piv, perm, tmp);
  }
}

template <int NB, int RMAX, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_blu_factor(Grid g, int mid, double2 *T, double2 *work) {
  extern __shared__ unsigned char smem[];
  blu_factor_body<NB, RMAX>(g, mid, MODE, blockIdx.x, T, work, smem);
}

template <typename R> __device__ inline cplx<R> to_r(double2 a) { return mk<R>((R)a.x, (R)a.y); }
template <typename R> __device__ inline cplx<R> to_r(float2 a) { return mk<R>((R)a.x, (R)a.y); }
template <typename IO> __device__ inline IO from_r(double2 a);
template <> __device__ inline double2 from_r<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_r<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <typename IO> __device__ inline IO from_r(float2 a);
template <> __device__ inline double2 from_r<double2>(float2 a) { return make_double2(a.x, a.y); }
template <> __device__ inline float2 from_r<float2>(float2 a) { return a; }

// y[s][j] = sum_l T_i[j][l] w[s][l] for the rows j = threadIdx.x < m.  The l-range is
// split over the blockDim.y wave groups (more loads in flight per column step); the
// partial sums meet in LDS and the complete result is valid in threads with
// threadIdx.y == 0.  Tt is T_i stored transposed, so lanes read consecutive rows.
template <typename R, int NS>
__device__ inline void col_matvec(const cplx<R> *__restrict__ Tt, int m, const cplx<R> *w, cplx<R> *part,
                                  cplx<R> (&acc)[NS]) {
  using C = cplx<R>;
  const int j = threadIdx.x, gy = threadIdx.y, G = blockDim.y;
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
  if (j < m) {
    const int chunk = (m + G - 1) / G;
    const int l0 = gy * chunk, l1 = min(m, l0 + chunk);
#pragma unroll 8
    for (int l = l0; l < l1; ++l) {
      C t = Tt[(size_t)l * m + j];
#pragma unroll
      for (int s = 0; s < NS; ++s) cfma(acc[s], t, w[s * m + l]);
    }
  }
  if (G > 1) {
    if (gy > 0 && j < m)
#pragma unroll
      for (int s = 0; s < NS; ++s) part[((gy - 1) * NS + s) * m + j] = acc[s];
    __syncthreads();
    if (gy == 0 && j < m)
      for (int q = 1; q < G; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = cadd(acc[s], part[((q - 1) * NS + s) * m + j]);
  }
}

// Forward sweeps: side 0 computes y_i for i = 0..mid-1, side 1 for i = nx-1..mid+1.
// T: factors of type cplx<R> ([nx][m][m], transposed); b, x: IO type [K][nz][nx].
// Block (roundup64(m), G): thread (j, 0) owns row j of every column vector.
template <typename R, typename IO, bool ADJ, int NS>
__device__ __forceinline__ void blu_fwd_body(const Grid &g, int K, int mid, const cplx<R> *__restrict__ T,
                                             const IO *b, IO *x, int group, int side, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *v = (C *)smem;          // [NS][m] previous y
  C *w = v + NS * m;         // [NS][m] right-hand side of this column
  C *part = w + NS * m;      // [G-1][NS][m] partial sums
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  const int cnt = side == 0 ? mid : g.nx - 1 - mid;
  auto col_of = [&](int step) { return side == 0 ? step : g.nx - 1 - step; };
  IO bnext[NS];
  if (owner && cnt > 0)
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (k0 + s < K) bnext[s] = b[(k0 + s) * Nu + (size_t)j * g.nx + col_of(0)];
  for (int step = 0; step < cnt; ++step) {
    const int i = col_of(step);
    const int cc = side == 0 ? i : i + 1;  // coupling column to the previous block
    if (owner) {
      C cj = step > 0 ? to_r<R>(coupling_x(g, cc, j)) : mk<R>(0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        C r = mk<R>(0, 0);
        if (k0 + s < K) {
          r = to_r<R>(bnext[s]);
          if (ADJ) r = cconj(r);
          if (step > 0) r = csub(r, cmul(cj, v[s * m + j]));
        }
        w[s * m + j] = r;
      }
      // prefetch the next column's right-hand side while the matvec runs
      if (step + 1 < cnt)
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (k0 + s < K) bnext[s] = b[(k0 + s) * Nu + (size_t)j * g.nx + col_of(step + 1)];
    }
    __syncthreads();
    C acc[NS];
    col_matvec<R, NS>(T + (size_t)i * mm, m, w, part, acc);
    if (owner) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        v[s * m + j] = acc[s];
        if (k0 + s < K) x[(k0 + s) * Nu + (size_t)j * g.nx + i] = from_r<IO>(acc[s]);
      }
    }
    __syncthreads();
  }
}

// Middle column: x_mid = T_mid (b_mid - C_mid y_{mid-1} - C_{mid+1} y_{mid+1}).
template <typename R, typename IO, bool ADJ, int NS>
__device__ __forceinline__ void blu_mid_body(const Grid &g, int K, int mid, const cplx<R> *__restrict__ T,
                                             const IO *b, IO *x, cplx<R> *xmid, int group, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *w = (C *)smem;
  C *part = w + 2 * NS * m;
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  if (owner) {
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
  C acc[NS];
  col_matvec<R, NS>(T + (size_t)mid * mm, m, w, part, acc);
  if (owner) {
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
__device__ __forceinline__ void blu_bwd_body(const Grid &g, int K, int mid, const cplx<R> *__restrict__ T, IO *x,
                                             const cplx<R> *xmid, int group, int side, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *w = (C *)smem;          // [NS][m] coupled previous x
  C *part = w + 2 * NS * m;
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const size_t Nu = (size_t)g.nx * g.nz;
  const size_t mm = (size_t)m * m;
  C xr[NS];
  if (owner)
#pragma unroll
    for (int s = 0; s < NS; ++s) xr[s] = (k0 + s < K) ? xmid[(size_t)(k0 + s) * m + j] : mk<R>(0, 0);
  const int cnt = side == 0 ? mid : g.nx - 1 - mid;
  for (int step = 0; step < cnt; ++step) {
    const int i = side == 0 ? mid - 1 - step : mid + 1 + step;
    const int cc = side == 0 ? i + 1 : i;
    IO yv[NS];
    if (owner) {
      C cj = to_r<R>(coupling_x(g, cc, j));
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        w[s * m + j] = cmul(cj, xr[s]);
        if (k0 + s < K) yv[s] = x[(k0 + s) * Nu + (size_t)j * g.nx + i];   // y_i, used after the matvec
      }
    }
    __syncthreads();
    C acc[NS];
    col_matvec<R, NS>(T + (size_t)i * mm, m, w, part, acc);
    if (owner) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (k0 + s < K) {
          C xi = csub(to_r<R>(yv[s]), acc[s]);
          xr[s] = xi;
          x[(k0 + s) * Nu + (size_t)j * g.nx + i] = from_r<IO>(ADJ ? cconj(xi) : xi);
        }
      }
    }
    __syncthreads();
  }
}

template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_fwd(Grid g, int K, int mid, const cplx<R> *__restrict__ T, const IO *b, IO *x) {
  extern __shared__ unsigned char smem[];
  blu_fwd_body<R, IO, ADJ, NS>(g, K, mid, T, b, x, blockIdx.x, blockIdx.y, smem);
}
template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_mid(Grid g, int K, int mid, const cplx<R> *__restrict__ T, const IO *b, IO *x, cplx<R> *xmid) {
  extern __shared__ unsigned char smem[];
  blu_mid_body<R, IO, ADJ, NS>(g, K, mid, T, b, x, xmid, blockIdx.x, smem);
}
template <typename R, typename IO, bool ADJ, int NS>
__global__ void k_blu_bwd(Grid g, int K, int mid, const cplx<R> *__restrict__ T, IO *x, const cplx<R> *xmid) {
  extern __shared__ unsigned char smem[];
  blu_bwd_body<R, IO, ADJ, NS>(g, K, mid, T, x, xmid, blockIdx.x, blockIdx.y, smem);
}

// ---------------------------------------------------------------------------
// Persistent work-list kernels for a batch of problems (several frequencies on
// uneven grids).  A fixed grid of workgroups drains one list of items covering every
// problem: a workgroup takes the next item index from a device counter, decodes
// (problem, source group, side) and runs the same body as the single-problem kernel.
// The loop ends for the whole workgroup at once when the list is exhausted, so every
// wave reaches the exit.  The counter is cleared by a kernel launched just before.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int next_item(unsigned int *counter, int *slot) {
  if (threadIdx.x == 0 && threadIdx.y == 0) *slot = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int item = *slot;
  __syncthreads();
  return item;
}

__device__ __forceinline__ int find_problem(const int *first, int nprob, int item) {
  int q = 0;
  while (q + 1 < nprob && first[q + 1] <= item) ++q;
  return q;
}

template <typename R, typename IO, bool ADJ, int NS, int PHASE>
__global__ void k_blu_sweep_batch(SweepBatch bt, unsigned int *counter) {
  extern __shared__ unsigned char smem[];
  __shared__ int slot;
  for (;;) {
    const int item = next_item(counter, &slot);
    if (item >= bt.total) break;
    const int q = find_problem(bt.first, bt.n, item);
    const SweepProblem &pp = bt.p[q];
    const int local = item - bt.first[q];
    const cplx<R> *T = (const cplx<R> *)pp.T;
    if (PHASE == 0)
      blu_fwd_body<R, IO, ADJ, NS>(pp.g, pp.K, pp.mid, T, (const IO *)pp.b, (IO *)pp.x, local >> 1, local & 1, smem);
    else if (PHASE == 1)
      blu_mid_body<R, IO, ADJ, NS>(pp.g, pp.K, pp.mid, T, (const IO *)pp.b, (IO *)pp.x, (cplx<R> *)pp.xmid, local, smem);
    else
      blu_bwd_body<R, IO, ADJ, NS>(pp.g, pp.K, pp.mid, T, (IO *)pp.x, (const cplx<R> *)pp.xmid, local >> 1, local & 1,
                                   smem);
    __syncthreads();
  }
}

template <int NB, int RMAX, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_blu_factor_batch(FactorBatch bt, unsigned int *counter) {
  extern __shared__ unsigned char smem[];
  __shared__ int slot;
  for (;;) {
    const int item = next_item(counter, &slot);
    if (item >= bt.total) break;
    const int q = find_problem(bt.first, bt.n, item);
    const FactorProblem &pp = bt.p[q];
    blu_factor_body<NB, RMAX>(pp.g, pp.mid, MODE, item - bt.first[q], pp.T, pp.work, smem);
    __syncthreads();
  }
}

__global__ void k_zero_u32(unsigned int *c) { *c = 0u; }

// block shape of the sweeps: x covers the rows, y splits each dot product
inline dim3 sweep_block(int m) {
  int rj = ((m + 63) / 64) * 64;
  int gy = 1024 / rj;
  gy = gy > 4 ? 4 : (gy < 1 ? 1 : gy);
  return dim3(rj, gy);
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
      Grid g = p->grid();
      auto launch = [&](auto sides, auto middle, int nb, int nthreads) -> kf_status {
        size_t smem = (2 * (size_t)m * nb + 2 * (size_t)m + 2 * nb) * sizeof(double2) + 2 * (size_t)m * sizeof(int);
        HIP_TRY(hipFuncSetAttribute((const void *)sides, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        HIP_TRY(hipFuncSetAttribute((const void *)middle, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        {
          ProfScope ps(p, PROF_FACTOR);
          hipLaunchKernelGGL(sides, dim3(2), dim3(nthreads), smem, p->stream, g, p->mid, p->T64, p->fac_work);
          LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(middle, dim3(1), dim3(nthreads), smem, p->stream, g, p->mid, p->T64, p->fac_work);
        LAUNCH_CHECK();
        return KF_OK;
      };
      // panel width and rows per lane of the register-resident panel, by column height
      // (the register-resident panel needs the larger VGPR budget of 256-thread groups
      //  once a lane owns five or more rows)
      kf_status st = m <= 128 ? launch(k_blu_factor<8, 2, 512, 0>, k_blu_factor<8, 2, 512, 1>, 8, 512)
                   : m <= 192 ? launch(k_blu_factor<8, 3, 512, 0>, k_blu_factor<8, 3, 512, 1>, 8, 512)
                   : m <= 320 ? launch(k_blu_factor<8, 5, 256, 0>, k_blu_factor<8, 5, 256, 1>, 8, 256)
                              : launch(k_blu_factor<8, 8, 256, 0>, k_blu_factor<8, 8, 256, 1>, 8, 256);
      if (st != KF_OK) return st;
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
  dim3 blk = sweep_block(m);
  size_t smem = (2 + (blk.y - 1)) * NS * m * sizeof(cplx<R>);
  const bool fp32 = sizeof(R) == sizeof(float);
  {
    ProfScope pf(p, fp32 ? PROF_FWD32 : PROF_FWD64);
    hipLaunchKernelGGL((k_blu_fwd<R, IO, ADJ, NS>), dim3(groups, 2), blk, smem, p->stream, g, p->K, p->mid, T, rhs, x);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_blu_mid<R, IO, ADJ, NS>), dim3(groups), blk, smem, p->stream, g, p->K, p->mid, T, rhs, x, xmid);
  LAUNCH_CHECK();
  {
    ProfScope pb(p, fp32 ? PROF_BWD32 : PROF_BWD64);
    hipLaunchKernelGGL((k_blu_bwd<R, IO, ADJ, NS>), dim3(groups, 2), blk, smem, p->stream, g, p->K, p->mid, T, x, xmid);
    LAUNCH_CHECK();
  }
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

// ---------------------------------------------------------------------------
// batch launchers: every problem of the batch in one persistent launch per phase
// ---------------------------------------------------------------------------
namespace {
template <int NB, int RMAX, int NT>
kf_status factor_batch_launch(const std::vector<kf_problem *> &ps, hipStream_t s, unsigned int *counter, int m_max) {
  FactorBatch bt{};
  bt.n = (int)ps.size();
  size_t smem = (2 * (size_t)m_max * NB + 2 * (size_t)m_max + 2 * NB) * sizeof(double2) + 2 * (size_t)m_max * sizeof(int);
  HIP_TRY(hipFuncSetAttribute((const void *)k_blu_factor_batch<NB, RMAX, NT, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  HIP_TRY(hipFuncSetAttribute((const void *)k_blu_factor_batch<NB, RMAX, NT, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  for (int mode = 0; mode < 2; ++mode) {
    int tot = 0;
    for (int q = 0; q < bt.n; ++q) {
      kf_problem *p = ps[q];
      bt.first[q] = tot;
      bt.p[q] = FactorProblem{p->grid(), p->mid, p->T64, p->fac_work};
      tot += mode == 0 ? 2 : 1;
    }
    bt.first[bt.n] = tot;
    bt.total = tot;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
    LAUNCH_CHECK();
    if (mode == 0) hipLaunchKernelGGL((k_blu_factor_batch<NB, RMAX, NT, 0>), dim3(tot), dim3(NT), smem, s, bt, counter);
    else hipLaunchKernelGGL((k_blu_factor_batch<NB, RMAX, NT, 1>), dim3(tot), dim3(NT), smem, s, bt, counter);
    LAUNCH_CHECK();
  }
  return KF_OK;
}
}  // namespace

kf_status blu_factor_batch(const std::vector<kf_problem *> &all, int which, hipStream_t s, unsigned int *counter) {
  std::vector<kf_problem *> ps;
  int m_max = 0;
  for (kf_problem *p : all)
    if ((which & 3) && !p->have_T64) { ps.push_back(p); m_max = std::max(m_max, p->nz); }
  if (!ps.empty()) {
    if ((int)ps.size() > KF_BATCH_MAX) { set_error("batch too large"); return KF_EINVAL; }
    kf_status st = m_max <= 128 ? factor_batch_launch<8, 2, 512>(ps, s, counter, m_max)
                 : m_max <= 192 ? factor_batch_launch<8, 3, 512>(ps, s, counter, m_max)
                 : m_max <= 320 ? factor_batch_launch<8, 5, 256>(ps, s, counter, m_max)
                                : factor_batch_launch<8, 8, 256>(ps, s, counter, m_max);
    if (st != KF_OK) return st;
    for (kf_problem *p : ps) p->have_T64 = true;
  }
  if (which & 2)
    for (kf_problem *p : all)
      if (!p->have_T32) {
        const size_t mm = (size_t)p->nz * p->nz;
        kf_status st = launch_copy_c128_to_c64(p, (int64_t)p->nx * mm, p->T64, p->T32);
        if (st != KF_OK) return st;
        p->have_T32 = true;
      }
  return KF_OK;
}

// rhs[q], x[q]: IO-typed fields of problem q; R = double uses the FP64 factors, float
// the complex64 ones.
template <typename R, typename IO>
kf_status blu_solve_batch(const std::vector<kf_problem *> &ps, int adjoint, const IO *const *rhs, IO *const *x,
                          hipStream_t s, unsigned int *counter) {
  constexpr int NS = 1;
  const bool fp32 = sizeof(R) == sizeof(float);
  SweepBatch bt{};
  bt.n = (int)ps.size();
  if (bt.n > KF_BATCH_MAX) { set_error("batch too large"); return KF_EINVAL; }
  int m_max = 0;
  for (int q = 0; q < bt.n; ++q) {
    kf_problem *p = ps[q];
    if (!(fp32 ? p->have_T32 : p->have_T64)) { set_error("batch solve before factorisation"); return KF_ESTATE; }
    m_max = std::max(m_max, p->nz);
    bt.p[q] = SweepProblem{p->grid(), p->K, p->mid, fp32 ? (const void *)p->T32 : (const void *)p->T64,
                           rhs[q], x[q], fp32 ? (void *)p->xmid32 : (void *)p->xmid};
  }
  dim3 blk = sweep_block(m_max);
  size_t smem = (2 + (blk.y - 1)) * NS * m_max * sizeof(cplx<R>);
  for (int phase = 0; phase < 3; ++phase) {
    int tot = 0;
    for (int q = 0; q < bt.n; ++q) {
      bt.first[q] = tot;
      const int groups = (ps[q]->K + NS - 1) / NS;
      tot += phase == 1 ? groups : 2 * groups;
    }
    bt.first[bt.n] = tot;
    bt.total = tot;
    const unsigned grid = (unsigned)std::min(tot, 1024);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
    LAUNCH_CHECK();
#define SWEEP_PHASE(PH)                                                                                     \
  if (adjoint) hipLaunchKernelGGL((k_blu_sweep_batch<R, IO, true, NS, PH>), dim3(grid), blk, smem, s, bt, counter); \
  else hipLaunchKernelGGL((k_blu_sweep_batch<R, IO, false, NS, PH>), dim3(grid), blk, smem, s, bt, counter);
    if (phase == 0) { SWEEP_PHASE(0) }
    else if (phase == 1) { SWEEP_PHASE(1) }
    else { SWEEP_PHASE(2) }
#undef SWEEP_PHASE
    LAUNCH_CHECK();
  }
  return KF_OK;
}
template kf_status blu_solve_batch<double, double2>(const std::vector<kf_problem *> &, int, const double2 *const *,
                                                    double2 *const *, hipStream_t, unsigned int *);
template kf_status blu_solve_batch<float, double2>(const std::vector<kf_problem *> &, int, const double2 *const *,
                                                   double2 *const *, hipStream_t, unsigned int *);
template kf_status blu_solve_batch<float, float2>(const std::vector<kf_problem *> &, int, const float2 *const *,
                                                  float2 *const *, hipStream_t, unsigned int *);
