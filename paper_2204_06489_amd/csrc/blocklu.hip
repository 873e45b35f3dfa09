// Block-tridiagonal LU of the 5-point Helmholtz operator over grid columns, in a
// partitioned form that keeps the whole GPU busy, and the batched forward / adjoint
// solves built on it.
//
// With unknowns grouped by grid column i (block size m = nz), A of Section 2 is
// block tridiagonal:  C_i x_{i-1} + D_i x_i + C_{i+1} x_{i+1} = b_i,
// D_i the (tridiagonal) column operator and C_i = diag(coupling of column i-1 and
// column i), the same in both directions because A is complex symmetric.
//
// Partition.  P - 1 separator columns s_1 < ... < s_{P-1} cut the columns into P
// chunks; chunk c holds the interior columns [a_c, b_c] and its meeting column mid_c.
// With the interior unknowns first, A = [A_II A_IS; A_SI A_SS], A_II block diagonal
// over chunks (each chunk block tridiagonal, Dirichlet at its separators).
//
// Factorisation (FP64):
//  1. every chunk: twisted LU from both ends, meeting at mid_c,
//       left   S_a = D_a,  S_i = D_i - C_i T_{i-1} C_i               a < i < mid
//       right  S_b = D_b,  S_i = D_i - C_{i+1} T_{i+1} C_{i+1}       mid < i < b
//       middle S_mid = D_mid - C_mid T_{mid-1} C_mid - C_{mid+1} T_{mid+1} C_{mid+1}
//     T_i = S_i^-1 (dense Gauss-Jordan with partial pivoting), stored transposed;
//  2. spikes: V^c = A_c^-1 E_a C_{a}  and  W^c = A_c^-1 E_b C_{b+1}, the chunk's
//     response to its left and right separator (m x m per column, by chunk solves
//     whose m right-hand sides are the coupling weights at one end column);
//  3. the reduced (Schur complement) system on the separators,
//       R_jj     = D_{s_j} - C_{s_j} W^{j-1}_{b} - C_{s_j+1} V^{j}_{a}
//       R_{j,j-1} = -C_{s_j} V^{j-1}_{b},   R_{j,j+1} = -C_{s_j+1} W^{j}_{a},
//     solved by block cyclic reduction: log2(P) levels, each eliminating every other
//     remaining separator at once (the blocks of each level sit in the separator
//     column's slots of T, V and W and in per-separator ML, MU arrays).
// Solve A x = b:
//  1. z = A_II^-1 b_I by the chunks' twisted sweeps (all chunks at once);
//  2. reduced right-hand side g_j = b_{s_j} - C_{s_j} z_{b} - C_{s_j+1} z_{a}, then
//     the separators' values by the reduction's forward levels, the root and the
//     back-substitution levels (one launch per level, all separators of a level and
//     all sources in parallel);
//  3. x_I = z - V x_{s_left} - W x_{s_right} (every interior column at once).
// P = 1 is the plain twisted LU of the whole grid.  The adjoint uses
// A^H = conj(A):  A^H x = b  <=>  A conj(x) = conj(b).
//
// Every source shares the factors, so one factorisation per (gamma, omega) serves
// all K forward and adjoint block solves of the stacked system (Section 2) and
// every preconditioner application (Section 5).
#include "common.h"

#include <cstring>
#include <type_traits>
#include <map>
#include <utility>
#include <vector>


namespace {

// Inversion of a batch of dense m x m blocks (the Schur complements of the chunk sweeps
// and the separators' pivot blocks) by Gauss-Jordan elimination with partial pivoting,
// in place on a row-major work matrix S, the inverse then written transposed.
//
// The columns are cut into blocks of GJ_NB; each elimination panel is one block.  The
// classical in-place steps on a panel (pivot row chosen over the rows not yet pivoted,
// interchanged, scaled; the pivot column eliminated from every other row and replaced
// by the accumulated transform) act on every other column x as
//     x  <-  (P x with the panel's pivot rows zeroed) + Pan (P x)[pivot rows],
// P the panel's row interchanges and Pan the finished panel: a rank-GJ_NB update.  One
// launch per panel, a workgroup per (column block, matrix): launch t applies panel t - 1
// to every other block, and the workgroup of block t, once its block is updated,
// eliminates panel t (its block) for the next launch.  So every column block of every
// matrix of the batch is updated in parallel, and the sequential pivot steps run on one
// workgroup per matrix, one panel per launch.  After the last panel the interchanges,
// composed into one row permutation, are undone on the columns.
//
// Behind each S (m x m double2) its integer staging: perm[2][m], the row permutation of
// the last two panels (perm[r] = the row whose content moved to r), and sig[2][m], the
// composition of every panel's interchanges so far.
constexpr int GJ_NB = 16;
constexpr int NB_MAX = 16;   // staging rows (double2) behind each work matrix

struct GjJob {
  int m;
  double2 *S;    // m x m row-major, followed by the integer staging
  double2 *Tt;   // destination: the inverse, transposed (T stored column-major)
};

// The pivot search compares 32-bit keys: the upper 22 bits of the modulus squared as an
// FP32 number (a non-negative float orders as its bit pattern; 13 mantissa bits are ample
// for choosing a pivot), then 1023 - row, so that the largest key is the largest modulus
// and, among equal ones, the lowest row.  NaN moduli, and rows already pivoted, get key
// 0; a key of 0 at the end means no finite entry (no interchange then).  Rows are
// below 512.
__device__ __forceinline__ unsigned gj_key(double a2, int r) {
  if (!(a2 == a2)) return 0u;
  const float f = a2 > 3.0e38 ? __builtin_inff() : (float)a2;
  return (__float_as_uint(f) & ~0x3FFu) | (unsigned)(1023 - r);
}

// One elimination step of a panel held one row per thread (acc: the row's NB panel
// entries): the pivot row chosen over the rows not yet pivoted (largest modulus, the
// lowest row on ties), exchanged with row k, scaled, and its column eliminated from
// every other row.  Q is a compile-time column, so acc stays in registers.
struct GjPanel {
  int r, m, k0, nw, lane, wave;
  bool row;
  double2 *cand;     // LDS [2][8][NB]: each wavefront's candidate pivot row, by step parity
  double2 *rowk;     // LDS [2][NB]: row k before the step
  unsigned *ckey;    // LDS [2][8]: each wavefront's best key
  int *lperm;        // LDS [m]: the panel's row permutation
};

// One barrier per step: every wavefront publishes its best key (and its row's values,
// and row k its values) before it, so that afterwards each thread finds the pivot row
// in LDS by itself.  The LDS areas alternate with the step's parity: a thread still
// reading step Q's areas cannot meet step Q + 1's writes, and step Q + 2's writes wait
// for the barrier of step Q + 1, which every thread reaches only after its reads of
// step Q.
template <int NB, int Q>
__device__ __forceinline__ void gj_pivot(const GjPanel &P, double2 (&acc)[NB]) {
  constexpr int PAR = Q & 1;
  const int k = P.k0 + Q;
  const unsigned mine = (P.row && P.r >= k) ? gj_key(cabs2(acc[Q]), P.r) : 0u;
  unsigned key = mine;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) key = max(key, (unsigned)__shfl_xor((int)key, o, 64));
  double2 *cand = P.cand + PAR * 8 * NB, *rowk = P.rowk + PAR * NB;
  if (P.lane == 0) P.ckey[PAR * 8 + P.wave] = key;
  if (key != 0u && mine == key)   // this wavefront's best row (keys are unique per row)
#pragma unroll
    for (int c = 0; c < NB; ++c) cand[P.wave * NB + c] = acc[c];
  if (P.r == k)
#pragma unroll
    for (int c = 0; c < NB; ++c) rowk[c] = acc[c];
  __syncthreads();
  unsigned best = 0u;
  int win = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w)
    if (w < P.nw) {
      const unsigned kw = P.ckey[PAR * 8 + w];
      if (kw > best) { best = kw; win = w; }
    }
  // a column with no finite entry leaves key 0: no interchange, every index stays in
  // range (the factors then carry the NaNs and the solves report them)
  const int bi = best != 0u ? 1023 - (int)(best & 0x3FFu) : P.m;
  const int pr = bi < P.m ? bi : k;
  const double2 *prow = bi < P.m ? cand + win * NB : rowk;
  if (P.r == 0) {
    const int tmp = P.lperm[k];
    P.lperm[k] = P.lperm[pr];
    P.lperm[pr] = tmp;
  }
  // the new row k is the old row pr, scaled; the pivot entry becomes 1 / pivot
  const double2 d = cdiv(make_double2(1.0, 0.0), prow[Q]);
  if (P.r == k) {
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = (c == Q) ? d : cmul(prow[c], d);
  } else if (P.row) {
    if (P.r == pr)   // the old row k moves to pr, then is eliminated like every other row
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] = rowk[c];
    // row -= (its entry in column Q) x the new row k = g x (old pivot row, 1 in column Q)
    const double2 g = cmul(acc[Q], d);
#pragma unroll
    for (int c = 0; c < NB; ++c)
      acc[c] = c == Q ? csub(make_double2(0.0, 0.0), g) : csub(acc[c], cmul(g, prow[c]));
  }
}

template <int NB, int Q> struct GjPivots {
  __device__ static __forceinline__ void run(const GjPanel &P, int ncol, double2 (&acc)[NB]) {
    if (Q < ncol) {   // uniform
      gj_pivot<NB, Q>(P, acc);
      GjPivots<NB, Q + 1>::run(P, ncol, acc);
    }
  }
};
template <int NB> struct GjPivots<NB, NB> {
  __device__ static __forceinline__ void run(const GjPanel &, int, double2 (&)[NB]) {}
};

// launch t of a batch inversion; grid (column blocks, matrices), one thread per row
// (blockDim.x >= m)
template <int NB>
__global__ __launch_bounds__(512) void k_gj_step(const GjJob *jobs, int t) {
  const GjJob J = jobs[blockIdx.y];
  const int m = J.m, npan = (m + NB - 1) / NB, b = blockIdx.x;
  const int pp = t - 1;                  // the panel this launch applies
  const bool fac = b == t;               // this block is the next panel
  if (b >= npan || !(fac || (pp >= 0 && pp < npan && b != pp))) return;   // uniform
  __shared__ double2 x1[NB][NB];
  __shared__ double2 cand[2][8][NB], rowk[2][NB];
  __shared__ unsigned ckey[2][8];
  __shared__ int lperm[512];
  int *perm = (int *)(J.S + (size_t)m * m), *sig = perm + 2 * m;
  const int r = threadIdx.x, nt = blockDim.x;
  const bool row = r < m;
  const int cb0 = b * NB, ncol = min(NB, m - cb0);
  double2 acc[NB];
  if (pp >= 0 && b != pp) {
    // the previous panel's interchanges and rank-nb update on this block
    const int K0 = pp * NB, nb = min(NB, m - K0);
    const int *pm = perm + (pp & 1) * m;
    for (int e = r; e < nb * NB; e += nt) {
      const int q = e / NB, c = e - q * NB;
      x1[q][c] = c < ncol ? J.S[(size_t)pm[K0 + q] * m + cb0 + c] : make_double2(0.0, 0.0);
    }
    if (row) {
      const bool piv_row = r >= K0 && r < K0 + nb;
      const double2 *src = J.S + (size_t)pm[r] * m + cb0;
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] = (!piv_row && c < ncol) ? src[c] : make_double2(0.0, 0.0);
    }
    __syncthreads();   // every read of the block's old rows before any write
    if (row) {
      const double2 *pan = J.S + (size_t)r * m + K0;
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < nb) {
          const double2 pq = pan[q];
#pragma unroll
          for (int c = 0; c < NB; ++c) cfma(acc[c], pq, x1[q][c]);
        }
    }
    if (!fac) {
      if (row)
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < ncol) J.S[(size_t)r * m + cb0 + c] = acc[c];
      return;
    }
  } else if (row) {
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = c < ncol ? J.S[(size_t)r * m + cb0 + c] : make_double2(0.0, 0.0);
  }
  // elimination of panel t (this block)
  for (int e = r; e < m; e += nt) lperm[e] = e;
  const GjPanel P{r, m, cb0, (nt + 63) >> 6, r & 63, r >> 6, row, &cand[0][0][0], &rowk[0][0], &ckey[0][0],
                  lperm};
  GjPivots<NB, 0>::run(P, ncol, acc);
  __syncthreads();   // lperm complete
  if (row)
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < ncol) J.S[(size_t)r * m + cb0 + c] = acc[c];
  int *pn = perm + (t & 1) * m;
  const int *sp = sig + ((t + 1) & 1) * m;
  int *sn = sig + (t & 1) * m;
  for (int e = r; e < m; e += nt) {
    const int o = lperm[e];
    pn[e] = o;
    sn[e] = t == 0 ? o : sp[o];   // content now at e came from original row sn[e]
  }
}

// after the last panel: Tt[c][j] = Sinv[j][c] = S[j][col(c)], col the inverse of the
// composed row permutation; 32 x 32 tiles through LDS, grid (tiles, matrices)
template <int NB>
__global__ __launch_bounds__(256) void k_gj_store(const GjJob *jobs) {
  const GjJob J = jobs[blockIdx.y];
  const int m = J.m, nt32 = (m + 31) / 32;
  if ((int)blockIdx.x >= nt32 * nt32) return;
  const int npan = (m + NB - 1) / NB;
  const int *sg = (const int *)(J.S + (size_t)m * m) + 2 * m + ((npan - 1) & 1) * m;
  __shared__ int col[512];
  __shared__ double2 tile[32][33];
  const int tid = threadIdx.x;
  for (int r = tid; r < m; r += 256) col[sg[r]] = r;
  __syncthreads();
  const int c0 = (blockIdx.x % nt32) * 32, j0 = (blockIdx.x / nt32) * 32;
  const int lo = tid & 31, hi = tid >> 5;
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // read S[j][col(c)] with lanes along c
    const int j = j0 + hi + 8 * p, c = c0 + lo;
    if (j < m && c < m) tile[lo][hi + 8 * p] = J.S[(size_t)j * m + col[c]];
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // write Tt[c][j] with lanes along j
    const int c = c0 + hi + 8 * p, j = j0 + lo;
    if (j < m && c < m) J.Tt[(size_t)c * m + j] = tile[hi + 8 * p][lo];
  }
}

// y[s][j] = sum_l T[j][l] w[s][l] for the rows j = threadIdx.x < m.  The l-range is
// split over the blockDim.y wave groups (more loads in flight per column step); the
// partial sums meet in LDS and the complete result is valid in threads with
// threadIdx.y == 0.  Tt is T stored transposed (column-major T), so lanes read
// consecutive rows.  A group walks its range in blocks of MV_U columns whose loads are
// all issued before the first use; the last block is padded (addresses clamped to the
// range, weights zero), so no element pays a load latency of its own.
// MV_U: 8 where many workgroups share the chip (their number hides the latency and
// fewer registers keep more of them resident), 16 on the sequential chains that only a
// few workgroups walk (every step's latency is exposed there).
template <typename R, int NS, int MV_U = 8>
__device__ inline void col_matvec(const cplx<R> *__restrict__ Tt, int m, const cplx<R> *w, cplx<R> *part,
                                  cplx<R> (&acc)[NS]) {
  using C = cplx<R>;
  const int j = threadIdx.x, gy = threadIdx.y, G = blockDim.y;
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
  const int chunk = (m + G - 1) / G;
  const int l0 = gy * chunk, l1 = min(m, l0 + chunk);
  const int jc = min(j, m - 1);   // rows past m compute a copy of row m - 1, never stored
  for (int lb = l0; lb < l1; lb += MV_U) {
    C t[MV_U];
#pragma unroll
    for (int u = 0; u < MV_U; ++u) t[u] = Tt[(size_t)min(lb + u, l1 - 1) * m + jc];
#pragma unroll
    for (int u = 0; u < MV_U; ++u) {
      const bool in = lb + u < l1;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const C wv = w[s * m + min(lb + u, l1 - 1)];
        cfma(acc[s], t[u], in ? wv : mk<R>(0, 0));
      }
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

// ---------------------------------------------------------------------------
// Work items.  One launch covers every item of every problem of a batch (a single
// problem is a batch of one).  Workgroups are dealt to the 8 XCDs in turn, so
// workgroup b runs on XCD b mod 8; XCD x is given the contiguous item range
// [xs[x], xs[x+1]), in launch order.  The host cuts the ranges at equal estimated cost
// (all items of one problem and phase cost about the same), so the XCDs finish
// together even when a batch mixes grids of very different size, and the items of
// one chunk (its source groups) share one XCD's L2 copy of the chunk's factors.
// Returns -1 for the workgroups past the end of their XCD's range.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int item_of_block(const int *xs) {
  const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
  const int it = xs[x] + r;
  return it < xs[x + 1] ? it : -1;
}

__device__ __forceinline__ int find_problem(const int *first, int nprob, int item) {
  int q = 0;
  while (q + 1 < nprob && first[q + 1] <= item) ++q;
  return q;
}

struct Chunk { int a, b, mid; };
// part: [P][3] = (a_c, b_c, mid_c); separator j (1..P-1) is column b_{j-1} + 1
__device__ __forceinline__ Chunk chunk_of(const int *part, int c) { return Chunk{part[3 * c], part[3 * c + 1], part[3 * c + 2]}; }
__device__ __forceinline__ int separator(const int *part, int j) { return part[3 * (j - 1) + 1] + 1; }

// ---------------------------------------------------------------------------
// factorisation kernels
// ---------------------------------------------------------------------------
// One Schur complement of the chunk sweeps, row-major into a work matrix:
//   S = D_i - C_a Tprev C_a (- C_b Tnext C_b)
// (ca, cb: the column whose coupling weights scale a correction, -1 for none; Tprev,
// Tnext stored transposed).
struct SchurJob {
  int q, i, ca, cb;            // problem of the batch, column, coupling columns
  const double2 *Tprev, *Tnext;
  double2 *S;
};

// grid (32 x 32 tiles, jobs); the transposed reads of T go through LDS
__global__ __launch_bounds__(256) void k_schur(FactorBatch bt, const SchurJob *jobs) {
  const SchurJob J = jobs[blockIdx.y];
  const Grid &g = bt.p[J.q].g;
  const int m = g.nz, nt32 = (m + 31) / 32;
  if ((int)blockIdx.x >= nt32 * nt32) return;
  const int l0 = (blockIdx.x % nt32) * 32, j0 = (blockIdx.x / nt32) * 32;
  __shared__ double2 ta[32][33], tb[32][33];
  const int tid = threadIdx.x, lo = tid & 31, hi = tid >> 5;
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // Tprev[j][l] = Tt[l][j], lanes along j
    const int l = l0 + hi + 8 * p, j = j0 + lo;
    if (l < m && j < m) {
      if (J.ca >= 0) ta[hi + 8 * p][lo] = J.Tprev[(size_t)l * m + j];
      if (J.cb >= 0) tb[hi + 8 * p][lo] = J.Tnext[(size_t)l * m + j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // S[j][l], lanes along l
    const int j = j0 + hi + 8 * p, l = l0 + lo;
    if (j >= m || l >= m) continue;
    double2 v = make_double2(0.0, 0.0);
    if (J.ca >= 0) v = csub(v, cmul(cmul(coupling_x(g, J.ca, j), ta[lo][hi + 8 * p]), coupling_x(g, J.ca, l)));
    if (J.cb >= 0) v = csub(v, cmul(cmul(coupling_x(g, J.cb, j), tb[lo][hi + 8 * p]), coupling_x(g, J.cb, l)));
    if (l >= j - 1 && l <= j + 1) {
      const Stencil5 st = stencil_at(g, J.i, j);
      v = cadd(v, l == j ? st.cc : (l < j ? st.czm : st.czp));
    }
    J.S[(size_t)j * m + l] = v;
  }
}

// Spike of chunk ch for the right-hand-side columns s0 .. s0+SP_N-1:
//   which 0: V = A_c^-1 E_a C_a     (unit coupling weights at column a)
//   which 1: W = A_c^-1 E_b C_{b+1} (at column b)
// by the chunk's twisted solve: forward from the loaded end to mid, the middle
// column, then back-substitution on both sides (the unloaded side's forward values
// are zero).  Out[i] holds the m x m block of column i, transposed like T.
// Each step is T_i times an m x SP_N block (SP_N = 16 columns of the spike): thread
// (row pair, half) owns rows 2 rp, 2 rp + 1 and columns 8 h .. 8 h + 7, so every element
// of T_i it reads feeds eight complex products and every LDS value two; a chunk's T_i
// are read m / 16 times per spike (from L2).  The step's right-hand side sits in LDS as
// [row][column]; the previous step's values are the thread's accumulators.
constexpr int SP_N = 16, SP_H = 8, SP_U = 4;
__host__ __device__ inline int spike_pairs_padded(int m) { return ((m + 1) / 2 + 63) / 64 * 64; }

__device__ __forceinline__ void spike_matvec(const double2 *__restrict__ Tt, int m, const double2 *w, int r0, int r1,
                                             int h, double2 (&acc)[2][SP_H]) {
#pragma unroll
  for (int s = 0; s < SP_H; ++s) acc[0][s] = acc[1][s] = make_double2(0.0, 0.0);
  const int r0c = min(r0, m - 1), r1c = min(r1, m - 1);
  for (int lb = 0; lb < m; lb += SP_U) {
    double2 ta[SP_U], tb[SP_U];
#pragma unroll
    for (int u = 0; u < SP_U; ++u) {
      const size_t row = (size_t)min(lb + u, m - 1) * m;
      ta[u] = Tt[row + r0c];
      tb[u] = Tt[row + r1c];
    }
#pragma unroll
    for (int u = 0; u < SP_U; ++u)
      if (lb + u < m) {
        const double2 *wl = w + (size_t)(lb + u) * SP_N + SP_H * h;
#pragma unroll
        for (int s = 0; s < SP_H; ++s) {
          const double2 wv = wl[s];
          cfma(acc[0][s], ta[u], wv);
          cfma(acc[1][s], tb[u], wv);
        }
      }
  }
}

__device__ __forceinline__ void spike_body(const Grid &g, Chunk ch, int which, int s0, const double2 *__restrict__ T,
                                           double2 *Out, double2 *w /* LDS [m][SP_N] */) {
  using C = double2;
  const int m = g.nz;
  const size_t mm = (size_t)m * m;
  // a batch launches the threads of its tallest grid: here threads past 2 RP (h > 1)
  // only take part in the barriers (their rows are out of range)
  const int RP = spike_pairs_padded(m);
  const int hh = threadIdx.x / RP, h = min(hh, 1), rp = hh > 1 ? m : threadIdx.x - hh * RP;
  const int rr[2] = {2 * rp, 2 * rp + 1};
  const int ecol = which == 0 ? ch.a : ch.b + 1;   // coupling column of the unit right-hand side
  const int rcol = which == 0 ? ch.a : ch.b;       // column it sits in
  C cur[2][SP_H];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < SP_H; ++t) cur[a][t] = make_double2(0.0, 0.0);
  // column s = s0 + 8 h + t of the unit right-hand side: the coupling weight at row s
  auto rhs = [&](int a, int t) {
    const int col = s0 + SP_H * h + t;
    return rr[a] == col && rr[a] < m ? coupling_x(g, ecol, rr[a]) : make_double2(0.0, 0.0);
  };
  auto put = [&](int a, int t, C v) { w[(size_t)rr[a] * SP_N + SP_H * h + t] = v; };
  auto store = [&](int i, C (&v)[2][SP_H]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
      if (rr[a] < m)
#pragma unroll
        for (int t = 0; t < SP_H; ++t) {
          const int col = s0 + SP_H * h + t;
          if (col < m) Out[(size_t)i * mm + (size_t)col * m + rr[a]] = v[a][t];
        }
  };
  auto load = [&](int i, C (&v)[2][SP_H]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int t = 0; t < SP_H; ++t) {
        const int col = s0 + SP_H * h + t;
        v[a][t] = rr[a] < m && col < m ? Out[(size_t)i * mm + (size_t)col * m + rr[a]] : make_double2(0.0, 0.0);
      }
  };
  // forward sweep from the loaded end
  const int fcnt = which == 0 ? ch.mid - ch.a : ch.b - ch.mid;
  for (int step = 0; step < fcnt; ++step) {
    const int i = which == 0 ? ch.a + step : ch.b - step;
    const int cc = which == 0 ? i : i + 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
      if (rr[a] < m) {
        const C cj = coupling_x(g, cc, rr[a]);
#pragma unroll
        for (int t = 0; t < SP_H; ++t) put(a, t, step == 0 ? rhs(a, t) : csub(make_double2(0.0, 0.0), cmul(cj, cur[a][t])));
      }
    __syncthreads();
    spike_matvec(T + (size_t)i * mm, m, w, rr[0], rr[1], h, cur);
    store(i, cur);
    __syncthreads();
  }
  // middle column
  {
    const int cc = which == 0 ? ch.mid : ch.mid + 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
      if (rr[a] < m) {
        const C cj = fcnt > 0 ? coupling_x(g, cc, rr[a]) : make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < SP_H; ++t) {
          C r = rcol == ch.mid ? rhs(a, t) : make_double2(0.0, 0.0);
          if (fcnt > 0) r = csub(r, cmul(cj, cur[a][t]));
          put(a, t, r);
        }
      }
  }
  __syncthreads();
  spike_matvec(T + (size_t)ch.mid * mm, m, w, rr[0], rr[1], h, cur);
  store(ch.mid, cur);
  __syncthreads();
  // back-substitution outward: x_i = y_i - T_i C x_prev (y_i = 0 on the unloaded side)
  for (int side = 0; side < 2; ++side) {
    const bool loaded = (side == 0) == (which == 0);
    const int cnt = side == 0 ? ch.mid - ch.a : ch.b - ch.mid;
    if (side == 1) load(ch.mid, cur);   // the middle values (written by this thread)
    for (int step = 0; step < cnt; ++step) {
      const int i = side == 0 ? ch.mid - 1 - step : ch.mid + 1 + step;
      const int cc = side == 0 ? i + 1 : i;
#pragma unroll
      for (int a = 0; a < 2; ++a)
        if (rr[a] < m) {
          const C cj = coupling_x(g, cc, rr[a]);
#pragma unroll
          for (int t = 0; t < SP_H; ++t) put(a, t, cmul(cj, cur[a][t]));
        }
      __syncthreads();
      C y[2][SP_H];
      if (loaded) load(i, y);
      spike_matvec(T + (size_t)i * mm, m, w, rr[0], rr[1], h, cur);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < SP_H; ++t) cur[a][t] = csub(loaded ? y[a][t] : make_double2(0.0, 0.0), cur[a][t]);
      store(i, cur);
      __syncthreads();
    }
  }
}

// item = (spike job, tile of SP_N columns); jobs 0..P-2: W of chunks 0..P-2, then V of
// chunks 1..P-1.
__global__ __launch_bounds__(512) void k_spikes(FactorBatch bt) {
  extern __shared__ unsigned char smem[];
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const FactorProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int gm = (pp.g.nz + SP_N - 1) / SP_N;
  const int job = local / gm, grp = local - job * gm;
  const int which = job < pp.P - 1 ? 1 : 0;
  const int c = which == 1 ? job : job - (pp.P - 1) + 1;
  spike_body(pp.g, chunk_of(pp.part, c), which, grp * SP_N, pp.T, which == 0 ? pp.V : pp.W, (double2 *)smem);
}

// ---- the separators' system by block cyclic reduction ----
// Separators j = 1..n (n = P - 1) carry the block-tridiagonal Schur complement
//   B_j = D_s - C_s W^{j-1}_b - C_{s+1} V^j_a,  L_j = -C_s V^{j-1}_b,  U_j = -C_{s+1} W^j_a
// (s = s_j; all m x m blocks column-major).  Level l eliminates the odd multiples of
// 2^l among the remaining separators, all at once: for such a j,
//   Binv_j = B_j^-1,  F_j = Binv_j L_j,  G_j = Binv_j U_j      (T, V, W slots of column s_j)
// and every even multiple k (neighbours j1 = k - 2^l, j2 = k + 2^l) becomes
//   B_k -= L_k G_j1 + U_k F_j2,  L_k <- -L_k F_j1,  U_k <- -U_k G_j2,
// with ML_k = L_k Binv_j1 and MU_k = U_k Binv_j2 kept for the right-hand side.  The last
// separator left, 2^top with top = floor(log2 n), is inverted at the end.
// A solve reduces g_k -= ML_k g_j1 + MU_k g_j2 level by level, takes x_root = Binv g,
// and substitutes back x_j = Binv_j g_j - F_j x_j1' - G_j x_j2' from the top level down:
// 2 top + 1 launches whose work within a level is all parallel.
constexpr int CR_LV = 6;   // levels: n <= 63

// one job of the factorisation's batched steps (pointers into the problems' buffers)
struct CrJob {
  int m;
  double alpha;
  const double2 *X, *Y, *Cin;
  double2 *Z;
};

// B_j, L_j, U_j of every separator of every problem; item = (problem, separator), the
// m x m entries grid-strided over blockIdx.x.  L, U: [n][4][m][m] (L, U, and two
// staging blocks for the next level's L, U).
__global__ void k_cr_setup(FactorBatch bt) {
  const int q = find_problem(bt.first, bt.n, blockIdx.y);
  const FactorProblem &pp = bt.p[q];
  const int j = blockIdx.y - bt.first[q] + 1, n = pp.P - 1;
  const Grid &g = pp.g;
  const int m = g.nz;
  const size_t mm = (size_t)m * m;
  const int s = separator(pp.part, j);
  double2 *B = pp.T + (size_t)s * mm;
  double2 *L = pp.lu + (size_t)(j - 1) * 4 * mm, *U = L + mm;
  const double2 *Wb = pp.W + (size_t)(s - 1) * mm, *Va = pp.V + (size_t)(s + 1) * mm;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < mm; e += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(e / m), r = (int)(e % m);   // entry (r, l), column-major
    const double2 cs = coupling_x(g, s, r), cs1 = coupling_x(g, s + 1, r);
    double2 v = csub(csub(make_double2(0.0, 0.0), cmul(cs, Wb[e])), cmul(cs1, Va[e]));
    if (l >= r - 1 && l <= r + 1) {
      const Stencil5 st = stencil_at(g, s, r);
      v = cadd(v, l == r ? st.cc : (l < r ? st.czm : st.czp));
    }
    B[e] = v;
    L[e] = j >= 2 ? csub(make_double2(0.0, 0.0), cmul(cs, pp.V[(size_t)(s - 1) * mm + e])) : make_double2(0.0, 0.0);
    U[e] = j <= n - 1 ? csub(make_double2(0.0, 0.0), cmul(cs1, pp.W[(size_t)(s + 1) * mm + e])) : make_double2(0.0, 0.0);
  }
}

// Z = Cin + alpha X Y (Cin may be NULL; Z may be Cin), column-major m x m; blockIdx.y =
// job.  32 x 32 output tile per workgroup, k in slabs of 16 through LDS; each of the
// 256 threads owns a 2 x 2 block of the tile.
__global__ __launch_bounds__(256) void k_cr_gemm(const CrJob *jobs) {
  const CrJob J = jobs[blockIdx.y];
  const int m = J.m;
  const int nt = (m + 31) / 32;
  if ((int)blockIdx.x >= nt * nt) return;
  const int r0 = (blockIdx.x % nt) * 32, c0 = (blockIdx.x / nt) * 32;
  __shared__ double2 xs[16][33], ys[16][33];
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  double2 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < m; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = t + 256 * u;
      {  // X[r0 + rr][k0 + kk] (column-major: contiguous in rr)
        const int kk = e >> 5, rr = e & 31;
        const int r = r0 + rr, k = k0 + kk;
        xs[kk][rr] = (r < m && k < m) ? J.X[(size_t)k * m + r] : make_double2(0.0, 0.0);
      }
      {  // Y[k0 + kk][c0 + cc] (contiguous in kk)
        const int cc = e >> 4, kk = e & 15;
        const int c = c0 + cc, k = k0 + kk;
        ys[kk][cc] = (c < m && k < m) ? J.Y[(size_t)c * m + k] : make_double2(0.0, 0.0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double2 x0 = xs[kk][tr], x1 = xs[kk][tr + 16];
      const double2 y0 = ys[kk][tc], y1 = ys[kk][tc + 16];
      cfma(acc[0][0], x0, y0);
      cfma(acc[0][1], x0, y1);
      cfma(acc[1][0], x1, y0);
      cfma(acc[1][1], x1, y1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int r = r0 + tr + 16 * a, c = c0 + tc + 16 * b;
      if (r < m && c < m) {
        const size_t o = (size_t)c * m + r;
        double2 v = cscale(acc[a][b], J.alpha);
        if (J.Cin) v = cadd(J.Cin[o], v);
        J.Z[o] = v;
      }
    }
}

// Z = X (X NULL: zero), m x m blocks; with alpha != 0 Z is row-major X (X column-major),
// the form the inversion kernel reads.  blockIdx.y = job.
__global__ void k_cr_copy(const CrJob *jobs) {
  const CrJob J = jobs[blockIdx.y];
  const size_t mm = (size_t)J.m * J.m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < mm; e += (size_t)gridDim.x * blockDim.x) {
    if (!J.X) { J.Z[e] = make_double2(0.0, 0.0); continue; }
    if (J.alpha != 0.0) {
      const int r = (int)(e / J.m), c = (int)(e % J.m);   // Z[r][c] = X[r][c] (X column-major)
      J.Z[e] = J.X[(size_t)c * J.m + r];
    } else {
      J.Z[e] = J.X[e];
    }
  }
}

// up to 1024 threads (4 wave groups of 256 rows) where the register budget allows
template <typename R, int NS> struct SolveThreads { static constexpr int N = sizeof(R) == 4 && NS <= 2 ? 1024 : 512; };
// sources per workgroup in the separators' reduction, given the sweeps' NS
template <typename R, int NS> struct CrSources { static constexpr int N = NS; };
template <typename R, int NS> struct SolveThreadsCR { static constexpr int N = SolveThreads<R, NS>::N; };

// ---------------------------------------------------------------------------
// solve phases.  They work in place on a column-major copy X of the right-hand
// sides ([K][nx][nz], compute type: column i of source k is X + (k nx + i) m), so a
// workgroup reads and writes whole columns with consecutive lanes.  The copy is
// made and undone by the transposes below; solves of A^H conjugate there
// (A^H x = b  <=>  A conj(x) = conj(b)), so the phases only ever solve with A.
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ cplx<R> *colp(void *X, const Grid &g, int k, int i) {
  return (cplx<R> *)X + ((size_t)k * g.nx + i) * g.nz;
}

// 0: chunk forward sweeps, item (chunk, side, group): side 0 computes y_i for
//    i = a..mid-1, side 1 for i = b..mid+1
template <typename R, int NS>
__device__ __forceinline__ void fwd_body(const Grid &g, int K, Chunk ch, const cplx<R> *__restrict__ T, void *X,
                                         int group, int side, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *w = (C *)smem;          // [NS][m] right-hand side of this column
  C *part = w + 2 * NS * m;  // [G-1][NS][m] partial sums
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const size_t mm = (size_t)m * m;
  const int cnt = side == 0 ? ch.mid - ch.a : ch.b - ch.mid;
  auto col_of = [&](int step) { return side == 0 ? ch.a + step : ch.b - step; };
  C prev[NS], bnext[NS];
  if (owner && cnt > 0)
#pragma unroll
    for (int s = 0; s < NS; ++s) bnext[s] = k0 + s < K ? colp<R>(X, g, k0 + s, col_of(0))[j] : mk<R>(0, 0);
  for (int step = 0; step < cnt; ++step) {
    const int i = col_of(step);
    const int cc = side == 0 ? i : i + 1;  // coupling column to the previous block
    if (owner) {
      const C cj = step > 0 ? ccast<R>(coupling_x(g, cc, j)) : mk<R>(0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        C r = bnext[s];
        if (step > 0) r = csub(r, cmul(cj, prev[s]));
        w[s * m + j] = r;
      }
      // prefetch the next column's right-hand side while the matvec runs
      if (step + 1 < cnt)
#pragma unroll
        for (int s = 0; s < NS; ++s)
          bnext[s] = k0 + s < K ? colp<R>(X, g, k0 + s, col_of(step + 1))[j] : mk<R>(0, 0);
    }
    __syncthreads();
    C acc[NS];
    col_matvec<R, NS>(T + (size_t)i * mm, m, w, part, acc);
    if (owner) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        prev[s] = acc[s];
        if (k0 + s < K) colp<R>(X, g, k0 + s, i)[j] = acc[s];
      }
    }
    __syncthreads();
  }
}

// 1: middle column of each chunk, x_mid = T_mid (b_mid - C_mid y_{mid-1} - C_{mid+1} y_{mid+1})
template <typename R, int NS>
__device__ __forceinline__ void mid_body(const Grid &g, int K, Chunk ch, const cplx<R> *__restrict__ T, void *X,
                                         int group, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *w = (C *)smem;
  C *part = w + 2 * NS * m;
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const int i = ch.mid;
  if (owner) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int k = k0 + s;
      C r = mk<R>(0, 0);
      if (k < K) {
        r = colp<R>(X, g, k, i)[j];
        if (i > ch.a) r = csub(r, cmul(ccast<R>(coupling_x(g, i, j)), colp<R>(X, g, k, i - 1)[j]));
        if (i < ch.b) r = csub(r, cmul(ccast<R>(coupling_x(g, i + 1, j)), colp<R>(X, g, k, i + 1)[j]));
      }
      w[s * m + j] = r;
    }
  }
  __syncthreads();
  C acc[NS];
  col_matvec<R, NS>(T + (size_t)i * m * m, m, w, part, acc);
  if (owner)
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (k0 + s < K) colp<R>(X, g, k0 + s, i)[j] = acc[s];
}

// 2: back-substitution outward from the middle: side 0: x_i = y_i - T_i C_{i+1} x_{i+1}
//    (i = mid-1..a); side 1: x_i = y_i - T_i C_i x_{i-1} (i = mid+1..b)
template <typename R, int NS>
__device__ __forceinline__ void bwd_body(const Grid &g, int K, Chunk ch, const cplx<R> *__restrict__ T, void *X,
                                         int group, int side, unsigned char *smem) {
  using C = cplx<R>;
  const int m = g.nz;
  C *w = (C *)smem;          // [NS][m] coupled previous x
  C *part = w + 2 * NS * m;
  const int j = threadIdx.x;
  const bool owner = threadIdx.y == 0 && j < m;
  const int k0 = group * NS;
  const size_t mm = (size_t)m * m;
  const int cnt = side == 0 ? ch.mid - ch.a : ch.b - ch.mid;
  C xr[NS];
  if (owner && cnt > 0)
#pragma unroll
    for (int s = 0; s < NS; ++s) xr[s] = k0 + s < K ? colp<R>(X, g, k0 + s, ch.mid)[j] : mk<R>(0, 0);
  for (int step = 0; step < cnt; ++step) {
    const int i = side == 0 ? ch.mid - 1 - step : ch.mid + 1 + step;
    const int cc = side == 0 ? i + 1 : i;
    C yv[NS];
    if (owner) {
      const C cj = ccast<R>(coupling_x(g, cc, j));
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        w[s * m + j] = cmul(cj, xr[s]);
        yv[s] = k0 + s < K ? colp<R>(X, g, k0 + s, i)[j] : mk<R>(0, 0);
      }
    }
    __syncthreads();
    C acc[NS];
    col_matvec<R, NS>(T + (size_t)i * mm, m, w, part, acc);
    if (owner) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        xr[s] = csub(yv[s], acc[s]);
        if (k0 + s < K) colp<R>(X, g, k0 + s, i)[j] = xr[s];
      }
    }
    __syncthreads();
  }
}

// 3: right-hand side of separator j, g_j = b_s - C_s z_{s-1} - C_{s+1} z_{s+1}, stored at
//    column s
template <typename R, int NS>
__device__ __forceinline__ void red_rhs_body(const Grid &g, int K, int s_col, void *X, int group) {
  using C = cplx<R>;
  const int m = g.nz;
  const int j = threadIdx.x;
  if (threadIdx.y != 0 || j >= m) return;
  const int k0 = group * NS;
  const C cl = ccast<R>(coupling_x(g, s_col, j)), cr = ccast<R>(coupling_x(g, s_col + 1, j));
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (k0 + s < K) {
      C r = colp<R>(X, g, k0 + s, s_col)[j];
      r = csub(r, cmul(cl, colp<R>(X, g, k0 + s, s_col - 1)[j]));
      r = csub(r, cmul(cr, colp<R>(X, g, k0 + s, s_col + 1)[j]));
      colp<R>(X, g, k0 + s, s_col)[j] = r;
    }
}

// 4: one level of the separators' cyclic reduction for NS sources: the value at column
//    out is set to (keep ? old value : 0) + M_0 x(col_0) - M_1 x(col_1) - M_2 x(col_2),
//    absent terms (NULL M_t) skipped.  A level is a handful of matvecs per workgroup, so
//    its cost is the depth of dependent loads: the workgroup is flat, thread t owning row
//    t mod m of column group t / m (up to 16 groups, 7 at m = 141 with 1024 threads), each
//    group walking a short range of every term's columns in blocks of 8 loads; the
//    signed vectors of all terms are staged in one round, and the terms accumulate into
//    one sum reduced once over the groups.
// pdst (not NULL): the sum is written there as [NS][m] instead of applied to column out
template <typename R, int NS>
__device__ __forceinline__ void cr_terms(const Grid &g, int K, void *X, int group, const cplx<R> *const *M,
                                         const int *col, int out, bool keep, unsigned char *smem,
                                         cplx<R> *pdst = nullptr) {
  using C = cplx<R>;
  constexpr int MV_U = 8;
  const int m = g.nz, nt = blockDim.x, tid = threadIdx.x;
  const int G = min(nt / m, 16);
  const int j = tid % m, gy = tid / m;
  const int k0 = group * NS;
  C *w = (C *)smem;            // [nterm][NS][m] signed vectors of the present terms
  C *part = w + 3 * NS * m;    // [G-1][NS][m] partial sums
  const C *Mc0 = M[0] ? M[0] : (M[1] ? M[1] : M[2]);
  const C *Mc1 = M[0] ? (M[1] ? M[1] : M[2]) : M[2];
  const C *Mc2 = M[2];
  const int cl0 = M[0] ? col[0] : (M[1] ? col[1] : col[2]);
  const int cl1 = M[0] ? (M[1] ? col[1] : col[2]) : col[2];
  const int cl2 = col[2];
  const int nterm = (M[0] != nullptr) + (M[1] != nullptr) + (M[2] != nullptr);
  const bool first_adds = M[0] != nullptr;   // term 0 adds, the others subtract
  for (int e = tid; e < nterm * NS * m; e += nt) {
    const int c = e / (NS * m), rem = e - c * NS * m, sidx = rem / m, r = rem - sidx * m;
    const int cl = c == 0 ? cl0 : c == 1 ? cl1 : cl2;
    const C v = k0 + sidx < K ? colp<R>(X, g, k0 + sidx, cl)[r] : mk<R>(0, 0);
    w[e] = (c == 0 && first_adds) ? v : mk<R>(-v.x, -v.y);
  }
  __syncthreads();
  C acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = mk<R>(0, 0);
  if (gy < G) {
    const int chunk = (m + G - 1) / G;
    const int l0 = gy * chunk, l1 = min(m, l0 + chunk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c >= nterm) break;   // uniform
      const C *Mt = c == 0 ? Mc0 : c == 1 ? Mc1 : Mc2;
      const C *wt = w + c * NS * m;
      for (int lb = l0; lb < l1; lb += MV_U) {
        C t[MV_U];
#pragma unroll
        for (int u = 0; u < MV_U; ++u) t[u] = Mt[(size_t)min(lb + u, l1 - 1) * m + j];
#pragma unroll
        for (int u = 0; u < MV_U; ++u) {
          const bool in = lb + u < l1;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const C wv = wt[s * m + min(lb + u, l1 - 1)];
            cfma(acc[s], t[u], in ? wv : mk<R>(0, 0));
          }
        }
      }
    }
  }
  if (G > 1) {
    if (gy > 0 && gy < G)
#pragma unroll
      for (int s = 0; s < NS; ++s) part[((gy - 1) * NS + s) * m + j] = acc[s];
    __syncthreads();
    if (gy == 0)
      for (int q = 1; q < G; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = cadd(acc[s], part[((q - 1) * NS + s) * m + j]);
  }
  if (gy == 0)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (pdst) pdst[s * m + j] = acc[s];
      else if (k0 + s < K) {
        C *d = colp<R>(X, g, k0 + s, out) + j;
        *d = keep ? cadd(*d, acc[s]) : acc[s];
      }
    }
}

__host__ __device__ inline int cr_top(int n) {   // floor(log2 n), n >= 1
  int t = 0;
  while ((2 << t) <= n) ++t;
  return t;
}

// KIND 0: forward reduction at level bt.level (item k = (t + 1) 2^(l+1)):
//           g_k -= ML_k g_{k-2^l} + MU_k g_{k+2^l};
// KIND 1: root, x = Binv g at separator 2^top;
// KIND 2: back-substitution at level bt.level (item j = (2t + 1) 2^l):
//           x_j = Binv_j g_j - F_j x_{j-2^l} - G_j x_{j+2^l}.
// The terms of kinds 0 and 2 go to workgroups of their own (a term slot each, so the
// chain of loads of each is one block's), which write their products as partials;
// k_cr_combine64 adds them in slot order and applies them.
// item = (separator, source group, term slot of the kind's split).
__host__ __device__ constexpr int cr_split64(int kind) { return kind == 0 ? 2 : kind == 2 ? 3 : 1; }
template <typename R, int NS, int KIND>
__global__ __launch_bounds__((SolveThreadsCR<R, NS>::N)) void k_cr_solve(SweepBatch bt) {
  extern __shared__ unsigned char smem[];
  using C = cplx<R>;
  constexpr int NTM = cr_split64(KIND);
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int G = (pp.K + NS - 1) / NS;
  const int tau = local % NTM, tile = local / NTM;
  const int grp = tile % G, t = tile / G;
  const Grid &g = pp.g;
  const int m = g.nz, n = pp.P - 1, lv = bt.level;
  const size_t mm = (size_t)m * m;
  const C *T = (const C *)pp.T, *V = (const C *)pp.V, *W = (const C *)pp.W, *CR = (const C *)pp.CR;
  // up to three terms at fixed slots (absent ones NULL)
  const C *M[3] = {nullptr, nullptr, nullptr};
  int col[3] = {0, 0, 0};
  int out;
  bool keep;
  if (KIND == 0) {
    const int st = 1 << lv, k = (t + 1) * 2 * st;
    out = separator(pp.part, k);
    keep = true;
    M[1] = CR + ((size_t)(k - 1) * CR_LV + lv) * 2 * mm;
    col[1] = separator(pp.part, k - st);
    if (k + st <= n) { M[2] = M[1] + mm; col[2] = separator(pp.part, k + st); }
  } else if (KIND == 1) {
    out = separator(pp.part, 1 << cr_top(n));
    keep = false;
    M[0] = T + (size_t)out * mm;
    col[0] = out;
  } else {
    const int st = 1 << lv, j = (2 * t + 1) * st;
    out = separator(pp.part, j);
    keep = false;
    M[0] = T + (size_t)out * mm;
    col[0] = out;
    if (j - st >= 1) { M[1] = V + (size_t)out * mm; col[1] = separator(pp.part, j - st); }
    if (j + st <= n) { M[2] = W + (size_t)out * mm; col[2] = separator(pp.part, j + st); }
  }
  if (NTM == 1) {
    cr_terms<R, NS>(g, pp.K, pp.x, grp, M, col, out, keep, smem);
    return;
  }
  // this workgroup's term: slot tau of a back-substitution, slot tau + 1 of a forward level
  const int slot = KIND == 0 ? tau + 1 : tau;
  if (!M[slot]) return;   // uniform: an edge separator has a term less
  const C *Ms[3] = {nullptr, nullptr, nullptr};
  Ms[slot] = M[slot];
  C *pdst = (C *)pp.crp + ((size_t)tile * 3 + slot) * NS * m;
  cr_terms<R, NS>(g, pp.K, pp.x, grp, Ms, col, out, keep, smem, pdst);
}

// The tiles of a split FP64 level: the partials of the present term slots added in slot
// order (the slots carry their signs) and applied: forward g_k += sum, back-substitution
// x_j = sum.  item = (separator, source group), blockIdx.x.
template <typename R, int NS, int KIND>
__global__ __launch_bounds__(256) void k_cr_combine64(SweepBatch bt) {
  using C = cplx<R>;
  const int item = blockIdx.x;
  if (item >= bt.total) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int tile = item - bt.first[q];
  const Grid &g = pp.g;
  const int m = g.nz, n = pp.P - 1, lv = bt.level, K = pp.K;
  const int G = (K + NS - 1) / NS;
  const int grp = tile % G, t = tile / G, st = 1 << lv;
  int out;
  bool has[3];
  if (KIND == 0) {
    const int k = (t + 1) * 2 * st;
    out = separator(pp.part, k);
    has[0] = false, has[1] = true, has[2] = k + st <= n;
  } else {
    const int j = (2 * t + 1) * st;
    out = separator(pp.part, j);
    has[0] = true, has[1] = j - st >= 1, has[2] = j + st <= n;
  }
  const C *part = (const C *)pp.crp + (size_t)tile * 3 * NS * m;
  for (int e = threadIdx.x; e < NS * m; e += 256) {
    const int s = e / m, j = e - s * m, k = grp * NS + s;
    C acc = mk<R>(0, 0);
    bool any = false;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (has[c]) {
        const C v = part[c * NS * m + e];
        acc = any ? cadd(acc, v) : v;
        any = true;
      }
    if (k < K) {
      C *d = colp<R>(pp.x, g, k, out) + j;
      *d = KIND == 0 ? cadd(*d, acc) : acc;
    }
  }
}

// 5: interior correction x_i = z_i - V_i x_{s_left} - W_i x_{s_right}.  Per chunk it is
// one dense product: with the interior columns of the chunk stacked (row R = (i - a) m
// + j), X_I -= [V_stack | W_stack] [x_{s_left}; x_{s_right}], an (L m) x 2m by 2m x K
// product, cut into CG_R x CG_S tiles (rows x sources).
constexpr int CG_R = 64, CG_S = 32;

// The interior correction of FP64 solves on the matrix cores: 64 x 32 tiles (rows of
// the chunk's stacked interior columns x sources, item = (chunk, row tile, source
// tile)), each wavefront 16 rows x 32 sources as two 16 x 16 tiles of
// v_mfma_f64_16x16x4f64 (four real products per complex one), k in slabs of CM_K
// through LDS with the next slab loaded while the current one is multiplied.  The
// f64 result layout (D[i][j] in lane j + 16 (i % 4), element i / 4) puts one lane's
// entries in four sources' columns, so the tile goes through LDS once more for
// row-contiguous updates.
constexpr int CM_K = 32;
__global__ __launch_bounds__(256) void k_correct64_mfma(SweepBatch bt) {
  using C = double2;
  typedef double dx4 __attribute__((ext_vector_type(4)));
  constexpr int SL = CM_K * (CG_R + 1) + CM_K * (CG_S + 1), TL = CG_S * (CG_R + 1);
  __shared__ C lds[SL > TL ? SL : TL];
  C(*As)[CG_R + 1] = (C(*)[CG_R + 1])lds;
  C(*Bs)[CG_S + 1] = (C(*)[CG_S + 1])(lds + CM_K * (CG_R + 1));
  C(*Out)[CG_R + 1] = (C(*)[CG_R + 1])lds;
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int stiles = (pp.K + CG_S - 1) / CG_S;
  const int st = local % stiles, rest = local / stiles;
  const int rtiles = (pp.lmax * pp.g.nz + CG_R - 1) / CG_R;
  const int c = rest / rtiles, rt = rest % rtiles;
  const Chunk ch = chunk_of(pp.part, c);
  const Grid &g = pp.g;
  const int m = g.nz, K = pp.K;
  const int rows = (ch.b - ch.a + 1) * m;
  const int R0 = rt * CG_R;
  if (R0 >= rows) return;   // uniform over the workgroup
  const size_t mm = (size_t)m * m;
  const bool hl = c > 0, hr = c < pp.P - 1;
  const int lk0 = hl ? 0 : m, lk1 = hr ? 2 * m : m;
  const C *V = (const C *)pp.V, *W = (const C *)pp.W;
  const int s0 = st * CG_S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NA = CM_K * CG_R / 256, NB = CM_K * CG_S / 256;
  // load slots: A element (row R0 + e % 64, k e / 64), B element (k e % CM_K, source
  // e / CM_K); rows past the chunk load a clamped address and are zeroed
  auto load_slab = [&](int kb, C (&ra)[NA], C (&rb)[NB]) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u, rr = e % CG_R, l = kb + e / CG_R;
      const int row = min(R0 + rr, rows - 1), lc = min(l, lk1 - 1);
      const size_t base = (size_t)(ch.a + row / m) * mm + (size_t)(lc < m ? lc : lc - m) * m + row % m;
      const C v = lc < m ? V[base] : W[base];
      ra[u] = (R0 + rr < rows && l < lk1) ? v : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u, l = kb + e % CM_K, sidx = s0 + e / CM_K;
      const int lc = min(l, lk1 - 1), k = min(sidx, K - 1);
      const C v = colp<double>(pp.x, g, k, lc < m ? ch.a - 1 : ch.b + 1)[lc < m ? lc : lc - m];
      rb[u] = (l < lk1 && sidx < K) ? v : make_double2(0.0, 0.0);
    }
  };
  dx4 re[2], im[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) re[y] = im[y] = dx4{0.0, 0.0, 0.0, 0.0};
  C ra[NA], rb[NB];
  load_slab(lk0, ra, rb);
  for (int kb = lk0; kb < lk1; kb += CM_K) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u;
      As[e / CG_R][e % CG_R] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      Bs[e % CM_K][e / CM_K] = rb[u];
    }
    __syncthreads();
    if (kb + CM_K < lk1) load_slab(kb + CM_K, ra, rb);   // in flight during the products
#pragma unroll
    for (int kq = 0; kq < CM_K / 4; ++kq) {
      const int kk = 4 * kq + (lane >> 4);
      const C a = As[kk][16 * wave + (lane & 15)];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const C b = Bs[kk][16 * y + (lane & 15)];
        re[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re[y], 0, 0, 0);
        re[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re[y], 0, 0, 0);
        im[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im[y], 0, 0, 0);
        im[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im[y], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // the tile to LDS as [source][row], then row-contiguous updates
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Out[16 * y + (lane & 15)][16 * wave + 4 * r + (lane >> 4)] = make_double2(re[y][r], im[y][r]);
  __syncthreads();
  constexpr int NE = CG_S * CG_R / 256;
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + 256 * u;
    const int sidx = e / CG_R, rr = e - sidx * CG_R;
    const int row = R0 + rr, k = s0 + sidx;
    if (row < rows && k < K) {
      C *d = colp<double>(pp.x, g, k, ch.a + row / m) + (row % m);
      *d = csub(*d, Out[sidx][rr]);
    }
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// The interior correction of complex64 solves with FP16 operands on the matrix cores.
// Each FP32 operand value v is scaled by a power of two and held as two FP16 numbers,
// hi = fp16(v') and lo = fp16(v' - hi), which carry 22 significant bits; a product is
// hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo lo term is below 2^-22 of it), three
// v_mfma_f32_16x16x32_f16 with FP32 accumulation, each eight times the k-depth of the
// FP32 instruction at half its cycles.  So the product keeps FP32-class accuracy
// while the matrix cores do a quarter of the work of the FP32 form, and the kernel is
// bound by reading the spikes (as many bytes as their complex64 copy).
// Scales: the spikes of interior column i (V_i and W_i together) by 2^e_i, the
// separator values of chunk c and source k (both separators together) by 2^f_ck, each
// bringing the largest modulus into [2^14, 2^15) so that hi stays finite and lo normal
// for all but the smallest entries; the result is scaled back by 2^-(e_i + f_ck).
// Split values (uint16 storage of FP16): [column][row j][k / 8][hi re, hi im, lo re,
// lo im][k % 8], k running over V_i's columns (0..m-1) then W_i's (mk..mk+m-1),
// zero-padded to mk = m rounded up to 32: the four parts of eight consecutive k sit in
// 64 contiguous bytes, so a k-step of 32 reads whole 128-byte lines of each row.
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
constexpr int CH_R = 128, CH_S = 48, CH_K = 32;

__device__ __forceinline__ int scale_exponent(float mx) {
  return mx > 0.f && mx <= 3.0e38f ? 14 - ilogbf(mx) : 0;
}

// chunk of column i (-1 for separator columns) and whether it has a left / right separator
__device__ __forceinline__ int interior_chunk(const int *part, int P, int i, bool &hl, bool &hr) {
  for (int c = 0; c < P; ++c)
    if (i >= part[3 * c] && i <= part[3 * c + 1]) {
      hl = c > 0;
      hr = c < P - 1;
      return c;
    }
  return -1;
}

// e_i for every column (block i): the largest |re|, |im| over V_i (with a left
// separator) and W_i (with a right one)
__global__ __launch_bounds__(256) void k_spike_exponents(Grid g, int P, const int *part, const float2 *V,
                                                         const float2 *W, int *vwe) {
  const int i = blockIdx.x, m = g.nz;
  const size_t mm = (size_t)m * m;
  bool hl = false, hr = false;
  const int c = interior_chunk(part, P, i, hl, hr);
  float mx = 0.f;
  if (c >= 0)
    for (size_t e = threadIdx.x; e < mm; e += 256) {
      if (hl) { const float2 v = V[(size_t)i * mm + e]; mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y))); }
      if (hr) { const float2 v = W[(size_t)i * mm + e]; mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y))); }
    }
  __shared__ float red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) vwe[i] = c >= 0 ? scale_exponent(red[0]) : 0;
}

// the split values of interior column blockIdx.y, a 32 x 32 tile (rows j, k) per workgroup
__global__ __launch_bounds__(256) void k_spike_split(Grid g, int P, const int *part, const float2 *V, const float2 *W,
                                                     const int *vwe, int k2, uint16_t *vwh) {
  const int i = blockIdx.y, m = g.nz, mk = k2 / 2;
  const size_t mm = (size_t)m * m;
  bool hl = false, hr = false;
  if (interior_chunk(part, P, i, hl, hr) < 0) return;
  const int jt = (m + 31) / 32;
  const int j0 = (blockIdx.x % jt) * 32, k0 = (blockIdx.x / jt) * 32;
  __shared__ float2 tile[32][33];
  const int lo = threadIdx.x & 31, hi = threadIdx.x >> 5;
  const int e = vwe[i];
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // read with lanes along j (column-major blocks)
    const int k = k0 + hi + 8 * p, j = j0 + lo;
    float2 v = make_float2(0.f, 0.f);
    if (j < m) {
      if (k < mk) { if (hl && k < m) v = V[(size_t)i * mm + (size_t)k * m + j]; }
      else if (hr && k - mk < m) v = W[(size_t)i * mm + (size_t)(k - mk) * m + j];
    }
    tile[hi + 8 * p][lo] = make_float2(ldexpf(v.x, e), ldexpf(v.y, e));
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p) {   // write with lanes along k
    const int j = j0 + hi + 8 * p, k = k0 + lo;
    if (j >= m || k >= k2) continue;
    const float2 v = tile[lo][hi + 8 * p];
    const _Float16 hr_ = (_Float16)v.x, hi_ = (_Float16)v.y;
    const _Float16 lr = (_Float16)(v.x - (float)hr_), li = (_Float16)(v.y - (float)hi_);
    const size_t o = ((size_t)i * m + j) * k2 * 4 + (size_t)(k >> 3) * 32 + (k & 7);
    vwh[o] = __builtin_bit_cast(uint16_t, hr_);
    vwh[o + 8] = __builtin_bit_cast(uint16_t, hi_);
    vwh[o + 16] = __builtin_bit_cast(uint16_t, lr);
    vwh[o + 24] = __builtin_bit_cast(uint16_t, li);
  }
}

// f_ck for every chunk c and source k of a solve: grid (K, P) of one batch problem
__global__ __launch_bounds__(256) void k_corr_exponents(SweepBatch bt) {
  const int q = find_problem(bt.first, bt.n, blockIdx.y);
  const SweepProblem &pp = bt.p[q];
  const int c = blockIdx.y - bt.first[q], k = blockIdx.x;
  if (k >= pp.K || pp.P < 2) return;
  const Chunk ch = chunk_of(pp.part, c);
  const int m = pp.g.nz;
  float mx = 0.f;
  for (int l = threadIdx.x; l < m; l += 256) {
    if (c > 0) { const float2 v = colp<float>(pp.x, pp.g, k, ch.a - 1)[l]; mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y))); }
    if (c < pp.P - 1) { const float2 v = colp<float>(pp.x, pp.g, k, ch.b + 1)[l]; mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y))); }
  }
  __shared__ float red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pp.corr_e[c * pp.K + k] = scale_exponent(red[0]);
}

// X_I -= [V | W] [x_{s_left}; x_{s_right}] per chunk: a 128 x 48 tile (rows x sources)
// per workgroup, each wavefront 32 rows (two 16-row tiles) x 3 source tiles; k in steps
// of 32: the separator values split into FP16 parts in LDS ([part][source][k], two
// buffers alternating with the k-step), the spikes' parts read by each lane straight
// from memory (eight consecutive k of its row: 64 contiguous bytes).
// Operand layout of v_mfma_f32_16x16x32_f16: A[i][k] in lane i + 16 (k / 8), element
// k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; D[i][j] in lane j + 16 (i / 4),
// element i % 4.  Products: re re and im im into their own sums (Re = rr - ii), the
// two cross products into a third (Im).  item = (chunk, row tile, source tile).
__global__ __launch_bounds__(256) void k_correct_h(SweepBatch bt) {
  using C = float2;
  constexpr int BK = CH_K + 8;   // LDS row of one source's k values (16-byte aligned)
  constexpr int BSZ = 2 * 4 * CH_S * BK * 2, OSZ = CH_S * (CH_R + 1) * 8;
  __shared__ __align__(16) unsigned char lds[BSZ > OSZ ? BSZ : OSZ];
  _Float16 *Bs = (_Float16 *)lds;                    // [2][4][CH_S][BK]
  C(*Out)[CH_R + 1] = (C(*)[CH_R + 1])lds;
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int K = pp.K, m = pp.g.nz, nx = pp.g.nx, k2 = pp.k2, mk = k2 / 2;
  const int stiles = (K + CH_S - 1) / CH_S;
  const int rtiles = (pp.lmax * m + CH_R - 1) / CH_R;
  const int st = local % stiles, rest = local / stiles;
  const int c = rest / rtiles, rt = rest % rtiles;
  const Chunk ch = chunk_of(pp.part, c);
  const int rows = (ch.b - ch.a + 1) * m;
  const int R0 = rt * CH_R;
  if (R0 >= rows) return;   // uniform over the workgroup
  const bool hl = c > 0, hr = c < pp.P - 1;
  const int kbeg = hl ? 0 : mk, kend = hr ? k2 : mk;
  const int s0 = st * CH_S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const C *xb = (const C *)pp.x;
  const int *ce = pp.corr_e + c * K;
  const _Float16 *H = (const _Float16 *)pp.vwh;
  // this lane's A rows (two tiles): column-stacked row R -> (column a + R / m, row R % m)
  const _Float16 *arow[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int R = min(R0 + wave * 32 + 16 * x + (lane & 15), rows - 1);
    arow[x] = H + ((size_t)(ch.a + R / m) * m + R % m) * k2 * 4 + 32 * (lane >> 4);
  }
  floatx4 rr[2][3], ii[2][3], im[2][3];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) rr[x][y] = ii[x][y] = im[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};
  // B staging: thread t < 4 CH_S converts eight consecutive k of source s0 + t / 4
  const int bsl = tid >> 2, bkg = (tid & 3) * 8, bsrc = s0 + bsl;
  const bool bact = tid < 4 * CH_S && bsrc < K;
  const int bf = bact ? ce[bsrc] : 0;
  // the next k-step's operands, loaded while the current one is multiplied
  halfx8 an[2][4];
  C bn[8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int p = 0; p < 4; ++p) an[x][p] = *(const halfx8 *)(arow[x] + 4 * k0 + 8 * p);
    const int part = k0 < mk ? 0 : 1, l0 = k0 - part * mk + bkg;
    const C *src = xb + ((size_t)(bact ? bsrc : 0) * nx + (part == 0 ? ch.a - 1 : ch.b + 1)) * m;
#pragma unroll
    for (int u = 0; u < 8; ++u) bn[u] = (bact && l0 + u < m) ? src[l0 + u] : make_float2(0.f, 0.f);
  };
  fetch(kbeg);
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += CH_K, buf ^= 1) {
    halfx8 a[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int p = 0; p < 4; ++p) a[x][p] = an[x][p];
    C bc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bc[u] = bn[u];
    // the next k-step's loads go out before this step's staging and barrier
    if (k0 + CH_K < kend) fetch(k0 + CH_K);
    _Float16 *Bb = Bs + buf * (4 * CH_S * BK);
    if (tid < 4 * CH_S) {   // separator values of this k-step, scaled and split
      halfx8 h[4];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float vr = ldexpf(bc[u].x, bf), vi = ldexpf(bc[u].y, bf);
        const _Float16 hr_ = (_Float16)vr, hi_ = (_Float16)vi;
        h[0][u] = hr_;
        h[1][u] = hi_;
        h[2][u] = (_Float16)(vr - (float)hr_);
        h[3][u] = (_Float16)(vi - (float)hi_);
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) *(halfx8 *)(Bb + (p * CH_S + bsl) * BK + bkg) = h[p];
    }
    // one barrier per k-step: the staging buffers alternate, so a wavefront that stages
    // step k + 1 cannot overwrite what a slower one still reads for step k, and the
    // buffer of step k + 2 is free once every wavefront has passed step k + 1's barrier
    __syncthreads();
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      halfx8 b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) b[p] = *(const halfx8 *)(Bb + (p * CH_S + 16 * y + (lane & 15)) * BK + 8 * (lane >> 4));
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        rr[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][0], b[0], rr[x][y], 0, 0, 0);
        rr[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][0], b[2], rr[x][y], 0, 0, 0);
        rr[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][2], b[0], rr[x][y], 0, 0, 0);
        ii[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][1], b[1], ii[x][y], 0, 0, 0);
        ii[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][1], b[3], ii[x][y], 0, 0, 0);
        ii[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][3], b[1], ii[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][0], b[1], im[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][0], b[3], im[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][2], b[1], im[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][1], b[0], im[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][1], b[2], im[x][y], 0, 0, 0);
        im[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x][3], b[0], im[x][y], 0, 0, 0);
      }
    }
  }
  __syncthreads();   // the output tile below reuses the staging buffers
  // tile to LDS as [source][row], scaled back, then column-contiguous updates
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr_ = wave * 32 + 16 * x + 4 * (lane >> 4) + r;
      const int R = min(R0 + rr_, rows - 1);
      const int ei = pp.vwe[ch.a + R / m];
#pragma unroll
      for (int y = 0; y < 3; ++y) {
        const int sidx = min(s0 + 16 * y + (lane & 15), K - 1);
        const int sc = -(ei + ce[sidx]);
        Out[16 * y + (lane & 15)][rr_] = make_float2(ldexpf(rr[x][y][r] - ii[x][y][r], sc), ldexpf(im[x][y][r], sc));
      }
    }
  __syncthreads();
  constexpr int NE = CH_S * CH_R / 256, EU = 8;
  static_assert(NE % EU == 0, "epilogue batches");
  C *xw = (C *)pp.x;
#pragma unroll 1
  for (int e0 = 0; e0 < NE; e0 += EU) {
    C *d[EU];
    C old[EU];
    bool ok[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = tid + 256 * (e0 + u);
      const int sidx = e / CH_R, rr_ = e - sidx * CH_R;
      const int row = R0 + rr_, k = s0 + sidx;
      ok[u] = row < rows && k < K;
      const int rc = min(row, rows - 1);
      d[u] = xw + ((size_t)min(k, K - 1) * nx + ch.a + rc / m) * m + (rc % m);
      old[u] = *d[u];
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = tid + 256 * (e0 + u);
      const int sidx = e / CH_R, rr_ = e - sidx * CH_R;
      const C o = Out[sidx][rr_];
      if (ok[u]) *d[u] = make_float2(old[u].x - o.x, old[u].y - o.y);
    }
  }
}

// The separators' reduction of complex64 solves on the matrix cores.  A level is, for
// each separator it writes, one product of its blocks [M_0 | M_1 | M_2] (m x nterm m,
// column-major) with the stacked vectors of the terms (nterm m x K) over every source,
// so a workgroup computes a 64 x 16 tile (rows x sources) of it with
// v_mfma_f32_16x16x4f32 (Gauss: three real products per complex one), each wavefront
// 16 rows, k in slabs of 64 through LDS with the next slab prefetched.  A level has
// few separators, so its time is the latency of one workgroup's chain of slabs: small
// tiles (many workgroups, few products each) beat wide ones here (64 x 48 tiles: 1.25x
// the time; 128- or 144-deep slabs: 1.07x and 1.2x).
// Each block is read once per 16 sources instead of once per source group of the
// vector-unit levels, and all rows of a level's separators run in parallel.  Tiles split a separator's rows over
// workgroups, so a back-substitution level (x_j = Binv_j g_j - F_j x_j1 - G_j x_j2,
// written over g_j) and the root take g_j from the copy staged by k_cr_stage instead
// of from the column they overwrite.
// The terms of a tile are split over workgroups (two for a forward level, three for a
// back-substitution level; the root has one), which shortens each chain of slabs to
// one block's: each writes its partial tile, and k_cr_combine adds the partials in
// term order and applies the update.  item = (separator, row tile, source tile, term).
constexpr int CRM_R = 64, CRM_S = 16, CRM_K = 64, CRM_ST = CRM_S / 16;
// workgroups per tile of a level of kind 0 (forward), 1 (root), 2 (back-substitution)
__host__ __device__ constexpr int cr_split(int kind) { return kind == 0 ? 2 : kind == 2 ? 3 : 1; }

// gsep[(j - 1) K + k][l] = the separator j column of source k, every separator
__global__ __launch_bounds__(256) void k_cr_stage(SweepBatch bt) {
  const int q = find_problem(bt.first, bt.n, blockIdx.y);
  const SweepProblem &pp = bt.p[q];
  const int col = blockIdx.y - bt.first[q];   // (separator - 1) K + source
  const int K = pp.K, j = col / K + 1, k = col - (j - 1) * K;
  const int m = pp.g.nz;
  const float2 *src = colp<float>(pp.x, pp.g, k, separator(pp.part, j));
  float2 *dst = (float2 *)pp.gsep + (size_t)col * m;
  for (int l = threadIdx.x; l < m; l += 256) dst[l] = src[l];
}

// slab loader of k_cr_mfma: a slab (CRM_K values of k from l0) lies in one term, whose
// block, source column (-1: the staged g_j) and sign the caller passes
template <int NA, int NB>
__device__ __forceinline__ void cr_load_slab(const float2 *Mt, int ct, float sg, const float2 *gj, const float2 *xb,
                                             int l0, int tid, int R0, int s0, int m, int K, int nx, float2 (&ra)[NA],
                                             float2 (&rb)[NB]) {
#pragma unroll
  for (int u = 0; u < NA; ++u) {   // A[R0 + rr][l0 + kk], coalesced over rows
    const int e = tid + 256 * u, rr = e % CRM_R, l = l0 + e / CRM_R;
    const int j = min(R0 + rr, m - 1);
    const float2 v = Mt[(size_t)min(l, m - 1) * m + j];
    ra[u] = (R0 + rr < m && l < m) ? v : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {   // B[l0 + kk][s0 + sidx], coalesced over k
    const int e = tid + 256 * u, l = l0 + e % CRM_K, sidx = s0 + e / CRM_K;
    const int lc = min(l, m - 1), k = min(sidx, K - 1);
    const float2 v = ct < 0 ? gj[(size_t)k * m + lc] : xb[((size_t)k * nx + ct) * m + lc];
    rb[u] = (l < m && sidx < K) ? make_float2(sg * v.x, sg * v.y) : make_float2(0.f, 0.f);
  }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_cr_mfma(SweepBatch bt) {
  using C = float2;
  constexpr int SLAB = CRM_K * (CRM_R + 2) + CRM_K * (CRM_S + 2), TILE = CRM_S * (CRM_R + 1);
  __shared__ C lds[SLAB > TILE ? SLAB : TILE];
  C(*As)[CRM_R + 2] = (C(*)[CRM_R + 2])lds;
  C(*Bs)[CRM_S + 2] = (C(*)[CRM_S + 2])(lds + CRM_K * (CRM_R + 2));
  C(*Out)[CRM_R + 1] = (C(*)[CRM_R + 1])lds;
  constexpr int NTM = cr_split(KIND);
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const Grid &g = pp.g;
  const int m = g.nz, K = pp.K, n = pp.P - 1, lv = bt.level;
  const int stiles = (K + CRM_S - 1) / CRM_S, rtiles = (m + CRM_R - 1) / CRM_R;
  const int tau = local % NTM, tile = local / NTM;   // this workgroup's term, its tile
  const int st = tile % stiles, rest = tile / stiles;
  const int rt = rest % rtiles, t = rest / rtiles;
  const size_t mm = (size_t)m * m;
  const C *T = (const C *)pp.T, *V = (const C *)pp.V, *W = (const C *)pp.W, *CR = (const C *)pp.CR;
  const C *gs = (const C *)pp.gsep;
  // up to three terms stacked along k: block, source column of x (-1: separator jg's
  // staged copy) and sign; named slots, so that nothing is indexed at run time
  const C *M0, *M1 = nullptr, *M2 = nullptr;
  int c0, c1 = 0, c2 = 0, jg = 0, nterm, out;
  float g0 = -1.f;
  bool keep;
  if (KIND == 0) {   // g_k -= ML_k g_{k - 2^l} + MU_k g_{k + 2^l}
    const int s2 = 1 << lv, k = (t + 1) * 2 * s2;
    out = separator(pp.part, k);
    keep = true;
    M0 = CR + ((size_t)(k - 1) * CR_LV + lv) * 2 * mm;
    c0 = separator(pp.part, k - s2);
    const bool right = k + s2 <= n;
    if (right) { M1 = M0 + mm; c1 = separator(pp.part, k + s2); }
    nterm = 1 + right;
  } else {           // x_j = Binv_j g_j (- F_j x_{j - 2^l} - G_j x_{j + 2^l})
    const int s2 = 1 << lv;
    const int j = KIND == 1 ? 1 << cr_top(n) : (2 * t + 1) * s2;
    out = separator(pp.part, j);
    keep = false;
    jg = j;
    M0 = T + (size_t)out * mm;
    c0 = -1;
    g0 = 1.f;
    const bool hf = KIND == 2 && j - s2 >= 1, hg = KIND == 2 && j + s2 <= n;
    const C *Fj = V + (size_t)out * mm, *Gj = W + (size_t)out * mm;
    const int cf = hf ? separator(pp.part, j - s2) : 0, cgc = hg ? separator(pp.part, j + s2) : 0;
    M1 = hf ? Fj : (hg ? Gj : nullptr);
    c1 = hf ? cf : cgc;
    M2 = hf && hg ? Gj : nullptr;
    c2 = cgc;
    nterm = 1 + hf + hg;
  }
  if (tau >= nterm) return;   // uniform: an edge separator has a term less
  const int R0 = rt * CRM_R, s0 = st * CRM_S, nx = g.nx;
  C *const xb = (C *)pp.x;   // column i of source k at xb + (k nx + i) m
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NA = CRM_K * CRM_R / 256, NB = CRM_K * CRM_S / 256;
  // each term's k range padded to a multiple of 4 (one MFMA k-step), cut into slabs;
  // this workgroup's: those of its term (of every term when the tile is not split)
  const int mp = (m + 3) / 4 * 4, spt = (mp + CRM_K - 1) / CRM_K;
  const int sl0 = NTM == 1 ? 0 : tau * spt, sl1 = NTM == 1 ? nterm * spt : sl0 + spt;
  const C *gj = gs + (size_t)(jg > 0 ? jg - 1 : 0) * K * m;
  auto load_slab = [&](int sl, C (&ra)[NA], C (&rb)[NB]) {
    const int tau = sl / spt, l0 = (sl - tau * spt) * CRM_K;   // uniform
    if (tau == 0) cr_load_slab(M0, c0, g0, gj, xb, l0, tid, R0, s0, m, K, nx, ra, rb);
    else if (tau == 1) cr_load_slab(M1, c1, -1.f, gj, xb, l0, tid, R0, s0, m, K, nx, ra, rb);
    else cr_load_slab(M2, c2, -1.f, gj, xb, l0, tid, R0, s0, m, K, nx, ra, rb);
  };
  floatx4 p1[CRM_ST], p2[CRM_ST], p3[CRM_ST];
#pragma unroll
  for (int y = 0; y < CRM_ST; ++y) p1[y] = p2[y] = p3[y] = floatx4{0.f, 0.f, 0.f, 0.f};
  C ra[NA], rb[NB];
  load_slab(sl0, ra, rb);
  for (int sl = sl0; sl < sl1; ++sl) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u;
      As[e / CRM_R][e % CRM_R] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      Bs[e % CRM_K][e / CRM_K] = rb[u];
    }
    __syncthreads();
    if (sl + 1 < sl1) load_slab(sl + 1, ra, rb);   // in flight during the products
    const int nkq = min(CRM_K, mp - (sl % spt) * CRM_K) / 4;   // k-steps of this slab
#pragma unroll
    for (int kq = 0; kq < CRM_K / 4; ++kq) {
      if (kq < nkq) {
        const int kk = 4 * kq + (lane >> 4);
        const C a = As[kk][wave * 16 + (lane & 15)];
        C b[CRM_ST];
#pragma unroll
        for (int y = 0; y < CRM_ST; ++y) b[y] = Bs[kk][16 * y + (lane & 15)];
        const float as = a.x + a.y;
#pragma unroll
        for (int y = 0; y < CRM_ST; ++y) {
          p1[y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[y].x, p1[y], 0, 0, 0);
          p2[y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[y].y, p2[y], 0, 0, 0);
          p3[y] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b[y].x + b[y].y, p3[y], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // tile to LDS as [source][row], then column-contiguous updates
#pragma unroll
  for (int y = 0; y < CRM_ST; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Out[16 * y + (lane & 15)][wave * 16 + 4 * (lane >> 4) + r] =
          make_float2(p1[y][r] - p2[y][r], p3[y][r] - p1[y][r] - p2[y][r]);
  __syncthreads();
  constexpr int NE = CRM_S * CRM_R / 256, TS = CRM_S * CRM_R;
  C o[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + 256 * u;
    o[u] = Out[e / CRM_R][e % CRM_R];
  }
  if (NTM > 1) {   // the partial of this term, for k_cr_combine
    C *part = pp.crp + ((size_t)tile * 3 + tau) * TS;
#pragma unroll
    for (int u = 0; u < NE; ++u) part[tid + 256 * u] = o[u];
    return;
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + 256 * u;
    const int sidx = e / CRM_R, rr = e - sidx * CRM_R;
    const int row = R0 + rr, k = s0 + sidx;
    if (row < m && k < K) {
      C *d = xb + ((size_t)k * nx + out) * m + row;
      *d = keep ? make_float2(d->x + o[u].x, d->y + o[u].y) : o[u];
    }
  }
}

// The tiles of a split level (kind 0 or 2): the partials of the separator's terms
// added in term order and applied (forward: g_k += sum; back-substitution: x_j = sum).
// item = (separator, row tile, source tile), one workgroup each, blockIdx.x.
template <int KIND>
__global__ __launch_bounds__(256) void k_cr_combine(SweepBatch bt) {
  using C = float2;
  const int item = blockIdx.x;
  if (item >= bt.total) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int tile = item - bt.first[q];
  const int m = pp.g.nz, K = pp.K, n = pp.P - 1, lv = bt.level, nx = pp.g.nx;
  const int stiles = (K + CRM_S - 1) / CRM_S, rtiles = (m + CRM_R - 1) / CRM_R;
  const int st = tile % stiles, rest = tile / stiles;
  const int rt = rest % rtiles, t = rest / rtiles;
  const int s2 = 1 << lv;
  int out, nterm;
  if (KIND == 0) {
    const int k = (t + 1) * 2 * s2;
    out = separator(pp.part, k);
    nterm = 1 + (k + s2 <= n);
  } else {
    const int j = (2 * t + 1) * s2;
    out = separator(pp.part, j);
    nterm = 1 + (j - s2 >= 1) + (j + s2 <= n);
  }
  constexpr int TS = CRM_S * CRM_R;
  const C *part = pp.crp + (size_t)tile * 3 * TS;
  C *const xb = (C *)pp.x;
  const int R0 = rt * CRM_R, s0 = st * CRM_S;
#pragma unroll
  for (int u = 0; u < TS / 256; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int sidx = e / CRM_R, rr = e - sidx * CRM_R;
    const int row = R0 + rr, k = s0 + sidx;
    C s = part[e];
    for (int w = 1; w < nterm; ++w) {
      const C v = part[w * TS + e];
      s = make_float2(s.x + v.x, s.y + v.y);
    }
    if (row < m && k < K) {
      C *d = xb + ((size_t)k * nx + out) * m + row;
      *d = KIND == 0 ? make_float2(d->x + s.x, d->y + s.y) : s;
    }
  }
}

// Chunk sweeps of complex64 solves on the matrix cores (columns up to 144 TPW rows).
// Item (chunk, side, tile of SW_S = 16 sources).  Each step is the product of the m x m
// block T_i with an m x 16 right-hand side, as v_mfma_f32_16x16x4f32 tiles.  The 9 TPW
// row tiles go to NW = 3 TPW wavefronts, SW_TW = 3 each (wave w: tiles w + NW x), and
// the launch bounds keep the registers within three waves per SIMD: two workgroups
// share a compute unit with three waves on every SIMD, where nine waves of one tile
// pair each would leave one workgroup per unit and three waves on one SIMD against
// two on the others.  Each tile keeps a ring of SW_D k-steps of T_i in registers, SW_D
// k-steps ahead of the products and into the next column at the end of a step (the
// blocks do not depend on the chain).
// A complex product is three real ones (Gauss):
//   P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi);  Re = P1 - P2,  Im = P3 - P1 - P2.
// Operand layout of the 16x16x4 instruction: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k, D[i][j] in lane j + 16 (i / 4), element i % 4.
// Per step: (a) thread r < 144 TPW, row r of all sixteen sources (coalesced over rows):
// store the previous column's result from LDS, form the right-hand side in LDS
// (forward: b_i - C y_prev; back-substitution: C x_prev, with y_i taking the place of
// the result it read; a chunk's middle, one step: b_mid - C_mid y_{mid-1} -
// C_{mid+1} y_{mid+1}); (b) each wave: its 16 x 16 tiles of T_i times the right-hand
// side, the result (forward and middle: the product; back-substitution: y_i - product)
// to LDS.
constexpr int SW_S = 16, SW_TW = 3;   // sources, row tiles per wave
template <int TPW> struct SweepShape {
  // rows, k-steps, waves, threads, ring depth (a divisor of KS: the ring's slot of a
  // k-step is then the same in every column)
  static constexpr int M = 144 * TPW, KS = M / 4, NW = 3 * TPW, NT = 64 * NW, D = TPW == 1 ? 9 : 8;
  static_assert(KS % D == 0, "ring depth divides the k-steps");
};
template <int PH, int TPW>   // PH 0: forward sweep, 1: chunk middles, 2: back-substitution
size_t sweep_mfma_lds() { return (size_t)2 * SweepShape<TPW>::M * (SW_S + 1) * sizeof(float2); }
template <int PH, int TPW>
__global__ __launch_bounds__(SweepShape<TPW>::NT, 3) void k_sweep_mfma(SweepBatch bt) {
  using C = float2;
  constexpr int SWM = SweepShape<TPW>::M, KS = SweepShape<TPW>::KS, NW = SweepShape<TPW>::NW;
  constexpr int SW_D = SweepShape<TPW>::D;
  static_assert(NW * SW_TW * 16 == SWM && SweepShape<TPW>::NT >= SWM, "tiles and phase (a) rows");
  extern __shared__ unsigned char smem_raw[];
  C(*Bv)[SW_S + 1] = (C(*)[SW_S + 1])smem_raw;   // right-hand side of the step (B operand)
  C(*Pv)[SW_S + 1] = Bv + SWM;                    // the previous column's result
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int ST = (pp.K + SW_S - 1) / SW_S;
  const int st = local % ST, rest = local / ST;
  // item: (chunk, side, source tile); the middles (PH 1) have no side
  const Chunk ch = chunk_of(pp.part, PH == 1 ? rest : rest >> 1);
  const int side = PH == 1 ? 0 : rest & 1;
  const Grid &g = pp.g;
  const int m = g.nz, K = pp.K, s0 = st * SW_S;
  const size_t mm = (size_t)m * m;
  const C *T = (const C *)pp.T;
  const int cnt = PH == 1 ? 1 : side == 0 ? ch.mid - ch.a : ch.b - ch.mid;
  if (cnt <= 0) return;   // uniform over the workgroup
  // column of step t and the coupling column to the previous one
  auto col_of = [&](int t) {
    return PH == 1 ? ch.mid
                   : PH == 0 ? (side == 0 ? ch.a + t : ch.b - t) : (side == 0 ? ch.mid - 1 - t : ch.mid + 1 + t);
  };
  auto cc_of = [&](int i) { return PH == 0 ? (side == 0 ? i : i + 1) : (side == 0 ? i + 1 : i); };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // phase (a) slots: the threads form four groups of SWM / 3, group q taking sources
  // 4 q .. 4 q + 3 and thread l of a group the rows l, l + SWM / 3, l + 2 SWM / 3
  // (coalesced over rows; rows from m on are zero in the right-hand side): slot u is
  // row block u / 4 and source 4 q + u % 4.  Per row block the coupling factor zn[row]
  // (-1 / h^2); the column's ixh[i] is uniform.
  constexpr int RB = SWM / 3, SA = 12;
  static_assert(4 * RB == SweepShape<TPW>::NT, "four source groups of SWM / 3 threads");
  const int sq = tid / RB, rb = tid % RB;
  const double ih2 = -1.0 / (g.h * g.h);
  int srow[3];
  C zf[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    srow[c] = rb + RB * c;
    const double2 z = g.zn[min(srow[c], m - 1)];
    zf[c] = make_float2((float)(z.x * ih2), (float)(z.y * ih2));
  }
  C *const Xb = (C *)pp.x;
  const size_t sstride = (size_t)g.nx * m;   // one source to the next
  auto slot_row = [&](int u) { return srow[u >> 2]; };
  auto slot_src = [&](int u) { return 4 * sq + (u & 3); };
  auto slot_ok = [&](int u) { return slot_row(u) < m && s0 + slot_src(u) < K; };
  // the column's address is uniform (scalar registers), the row the lane's offset
  auto xaddr = [&](int u, int i) {
    return (Xb + (size_t)min(s0 + slot_src(u), K - 1) * sstride + (size_t)i * m) + min(slot_row(u), m - 1);
  };
  // A operand of column i, tile x: lane (i', k') = (lane % 16, lane / 16) of k-step ks
  // holds T_i[16 (wave + NW x) + i'][4 ks + k'] (column-major block: rows contiguous).
  // Every wave runs all KS k-steps (rows past m are clamped to row m - 1, k-steps past
  // the last one repeat it: the right-hand side is zero there), so the loads are
  // unconditional and the wait counts stay exact across the loop.  The last k-step reads
  // up to three columns beyond the block: the next block, or the zero padding after the
  // last one.
  const int akq = lane >> 4;
  int arw[SW_TW];
#pragma unroll
  for (int x = 0; x < SW_TW; ++x) arw[x] = min(16 * (wave + NW * x) + (lane & 15), m - 1);
  const int ksl = (m - 1) / 4;
  // the loads as buffer loads: the block's descriptor in scalar registers (its range,
  // the block and the three columns after it, lies inside T's allocation), the lane's
  // offset in a vector register, the k-step's offset in a scalar one
  const int nrec = (int)((mm + 4 * (size_t)m) * sizeof(C)), kso = 4 * m * (int)sizeof(C);
  auto rsrc_of = [&](int i) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)(T + (size_t)i * mm), (short)0, nrec, 0x00020000);
  };
  int avo[SW_TW];
#pragma unroll
  for (int x = 0; x < SW_TW; ++x) avo[x] = (akq * m + arw[x]) * (int)sizeof(C);
  auto aload = [&](__amdgpu_buffer_rsrc_t rs, int x, int ks) {
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(rs, avo[x], min(ks, ksl) * kso, 0));
  };
  C areg[SW_D][SW_TW];
  // right-hand-side values of the next step, held in registers
  C bnext[SA];
  if (PH == 2) {   // x_mid into Pv
#pragma unroll
    for (int u = 0; u < SA; ++u) Pv[slot_row(u)][slot_src(u)] = slot_ok(u) ? *xaddr(u, ch.mid) : make_float2(0.f, 0.f);
    __syncthreads();
  }
  // in the loop's order: right-hand side, coupling factor, then the block
  {
    const int i0 = col_of(0);
#pragma unroll
    for (int u = 0; u < SA; ++u) bnext[u] = *xaddr(u, i0);
  }
  // coupling to the previous column: C_cc = zn[row] ixh[cc] (-1 / h^2); the column
  // factor of the next step is fetched with the next right-hand side, ahead of the
  // block's loads
  double2 xh = g.ixh[PH == 2 ? cc_of(col_of(0)) : col_of(0)];
  // the middle's neighbours y_{mid-1}, y_{mid+1} (PH 1; zero where the chunk has none),
  // read where the right-hand side is formed (the middle is a single step)
  const bool hl = PH == 1 && ch.mid > ch.a, hr = PH == 1 && ch.mid < ch.b;
  const double2 xh2 = PH == 1 ? g.ixh[ch.mid + 1] : make_double2(0.0, 0.0);
  {
    const __amdgpu_buffer_rsrc_t r0 = rsrc_of(col_of(0));
#pragma unroll
    for (int x = 0; x < SW_TW; ++x)
#pragma unroll
      for (int ks = 0; ks < SW_D; ++ks) areg[ks][x] = aload(r0, x, ks);
  }
  for (int t = 0; t < cnt; ++t) {
    const int i = col_of(t);
    const C xf = make_float2((float)xh.x, (float)xh.y);
    // (a) store the previous result, form this step's right-hand side
#pragma unroll
    for (int u = 0; u < SA; ++u) {
      const int r = slot_row(u), j = slot_src(u);
      const C z = zf[u >> 2];
      const C cj = make_float2(z.x * xf.x - z.y * xf.y, z.x * xf.y + z.y * xf.x);
      const C pv = Pv[r][j];
      if (t > 0 && slot_ok(u)) *xaddr(u, col_of(t - 1)) = pv;
      const C cp = make_float2(cj.x * pv.x - cj.y * pv.y, cj.x * pv.y + cj.y * pv.x);
      const C bv = bnext[u];
      C rhs;
      if (PH == 0) rhs = t > 0 ? make_float2(bv.x - cp.x, bv.y - cp.y) : bv;
      else if (PH == 1) {
        // b_mid - C_mid y_{mid-1} - C_{mid+1} y_{mid+1}
        const C xf2 = make_float2((float)xh2.x, (float)xh2.y);
        const C cr = make_float2(z.x * xf2.x - z.y * xf2.y, z.x * xf2.y + z.y * xf2.x);
        const C ym = hl ? *xaddr(u, ch.mid - 1) : make_float2(0.f, 0.f);
        const C yp = hr ? *xaddr(u, ch.mid + 1) : make_float2(0.f, 0.f);
        const C tl = make_float2(cj.x * ym.x - cj.y * ym.y, cj.x * ym.y + cj.y * ym.x);
        const C tr = make_float2(cr.x * yp.x - cr.y * yp.y, cr.x * yp.y + cr.y * yp.x);
        rhs = make_float2(bv.x - tl.x - tr.x, bv.y - tl.y - tr.y);
      } else {
        rhs = cp;
        Pv[r][j] = bv;   // y_i, read back by the lane that forms x_i after the barrier
      }
      Bv[r][j] = slot_ok(u) ? rhs : make_float2(0.f, 0.f);
    }
    if (t + 1 < cnt) {
      const int in = col_of(t + 1);
#pragma unroll
      for (int u = 0; u < SA; ++u) bnext[u] = *xaddr(u, in);
      xh = g.ixh[cc_of(in)];
    }
    __syncthreads();
    // (b) the wave's 16 x 16 tiles of T_i times the right-hand side (rows past m are
    //     copies of row m - 1, which nothing reads), the blocks fetched ahead as they
    //     are consumed (the last step fetches its own block again)
    {
      floatx4 p1[SW_TW], p2[SW_TW], p3[SW_TW];
#pragma unroll
      for (int x = 0; x < SW_TW; ++x) p1[x] = p2[x] = p3[x] = floatx4{0.f, 0.f, 0.f, 0.f};
      const __amdgpu_buffer_rsrc_t rc = rsrc_of(i), rn = rsrc_of(t + 1 < cnt ? col_of(t + 1) : i);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const C b = Bv[4 * ks + akq][lane & 15];
        const float bs = b.x + b.y;
#pragma unroll
        for (int x = 0; x < SW_TW; ++x) {
          const C a = areg[ks % SW_D][x];
          const float as = a.x + a.y;
          p1[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, p1[x], 0, 0, 0);
          p2[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, p2[x], 0, 0, 0);
          p3[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, bs, p3[x], 0, 0, 0);
          // refill: k-step ks + SW_D of this column, else of the next one
          const int kn = ks + SW_D;
          areg[ks % SW_D][x] = kn < KS ? aload(rc, x, kn) : aload(rn, x, kn - KS);
        }
        // keep each k-step's work in place: a sum of a later step's operands moved up
        // would wait for that step's load
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int x = 0; x < SW_TW; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + NW * x) + 4 * (lane >> 4) + r, j = lane & 15;   // row < SWM
          const C o = make_float2(p1[x][r] - p2[x][r], p3[x][r] - p1[x][r] - p2[x][r]);
          if (PH != 2) Pv[row][j] = o;
          else {   // x_i = y_i - T_i C x_prev
            const C y = Pv[row][j];
            Pv[row][j] = make_float2(y.x - o.x, y.y - o.y);
          }
        }
    }
    __syncthreads();
  }
  // the last column's result
  const int il = col_of(cnt - 1);
#pragma unroll
  for (int u = 0; u < SA; ++u)
    if (slot_ok(u)) *xaddr(u, il) = Pv[slot_row(u)][slot_src(u)];
}

// Spikes on the matrix cores (columns up to 144 TPW rows): the chain of k_spikes (the
// chunk's twisted solve for SP_N = 16 unit right-hand-side columns per item) with each
// step T_i (m x m) times the m x 16 block as v_mfma_f64_16x16x4f64 tiles, four real
// products per complex one.  Operand layout: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k as for the f32 16x16x4 instruction, but D[i][j] in lane j + 16 (i % 4),
// element i / 4 (unlike the f32 form's lane j + 16 (i / 4), element i % 4).  The row tiles are those of the complex64 sweeps (three per wave, 3 TPW waves).
// The coupling to the next column is diagonal in the rows, so the lanes that hold a
// step's result also form the next step's right-hand side: the B operand is the only
// LDS, and a step is (barrier, products, barrier, result and next right-hand side).
// The blocks come in through buffer loads, a ring of SPM_D k-steps ahead, whose range is
// the block: columns past m - 1 (the last k-steps, where the right-hand side is zero)
// read as zero, so no read leaves the block.  The lane's offset runs in a vector
// register, the range check covering all of it.
constexpr int SPM_D = 4;
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <int TPW> struct F64Chain {
  using C = double2;
  static constexpr int KS = SweepShape<TPW>::KS, NW = SweepShape<TPW>::NW;
  static_assert(KS % SPM_D == 0 && NW * SW_TW * 16 == SweepShape<TPW>::M, "ring slots and row tiles");
  const C *T;
  size_t mm;
  int nrec, kso, akq, jc;
  int avo[SW_TW], loff[SW_TW];   // the lane's offset in a block; the next k-step's, per tile
  C areg[SPM_D][SW_TW];
  // lane (i', k') of k-step ks reads T_i[16 (wave + NW x) + i'][4 ks + k']
  __device__ __forceinline__ void init(const C *T_, int m, int lane, int wave) {
    T = T_;
    mm = (size_t)m * m;
    nrec = (int)(mm * sizeof(C));
    kso = 4 * m * (int)sizeof(C);
    akq = lane >> 4;
    jc = lane & 15;
#pragma unroll
    for (int x = 0; x < SW_TW; ++x) avo[x] = (akq * m + min(16 * (wave + NW * x) + jc, m - 1)) * (int)sizeof(C);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int i) const {
    return __builtin_amdgcn_make_buffer_rsrc((void *)(T + (size_t)i * mm), (short)0, nrec, 0x00020000);
  }
  __device__ __forceinline__ C aload(__amdgpu_buffer_rsrc_t rs, int off) const {
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  }
  // the first SPM_D k-steps of column i0
  __device__ __forceinline__ void prime(int i0) {
    const __amdgpu_buffer_rsrc_t r0 = rsrc(i0);
#pragma unroll
    for (int x = 0; x < SW_TW; ++x) {
      loff[x] = avo[x];
#pragma unroll
      for (int ks = 0; ks < SPM_D; ++ks) {
        areg[ks][x] = aload(r0, loff[x]);
        loff[x] += kso;
      }
    }
  }
  // re + i im = T_i B for this wave's row tiles (B[k][j] = Bv[k][j]); the ring runs on
  // into column inext
  __device__ __forceinline__ void product(const C (*Bv)[SP_N + 1], int i, int inext, doublex4 (&re)[SW_TW],
                                          doublex4 (&im)[SW_TW]) {
#pragma unroll
    for (int x = 0; x < SW_TW; ++x) re[x] = im[x] = doublex4{0.0, 0.0, 0.0, 0.0};
    const __amdgpu_buffer_rsrc_t rc = rsrc(i), rn = rsrc(inext);
    // the offsets stay a running sum: without this the compiler keeps one register per
    // k-step and tile for the whole kernel
#pragma unroll
    for (int x = 0; x < SW_TW; ++x) asm volatile("" : "+v"(loff[x]));
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const C b = Bv[4 * ks + akq][jc];
#pragma unroll
      for (int x = 0; x < SW_TW; ++x) {
        const C a = areg[ks % SPM_D][x];
        re[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re[x], 0, 0, 0);
        re[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re[x], 0, 0, 0);
        im[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im[x], 0, 0, 0);
        im[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im[x], 0, 0, 0);
        if (ks + SPM_D == KS) loff[x] = avo[x];   // the next column's first k-step
        areg[ks % SPM_D][x] = aload(ks + SPM_D < KS ? rc : rn, loff[x]);
        loff[x] += kso;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
};
template <int TPW>
size_t f64_chain_lds() { return (size_t)SweepShape<TPW>::M * (SP_N + 1) * sizeof(double2); }
template <int TPW>
__global__ __launch_bounds__(SweepShape<TPW>::NT, 3) void k_spikes_mfma(FactorBatch bt) {
  using C = double2;
  constexpr int NW = SweepShape<TPW>::NW;
  extern __shared__ unsigned char smem_raw[];
  C(*Bv)[SP_N + 1] = (C(*)[SP_N + 1])smem_raw;
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const FactorProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const Grid &g = pp.g;
  const int m = g.nz;
  const size_t mm = (size_t)m * m;
  const int gm = (m + SP_N - 1) / SP_N;
  const int job = local / gm, grp = local - job * gm;
  const int which = job < pp.P - 1 ? 1 : 0;   // 1: W of chunk job, 0: V of chunk job - (P - 1) + 1
  const Chunk ch = chunk_of(pp.part, which == 1 ? job : job - (pp.P - 1) + 1);
  C *const Out = which == 0 ? pp.V : pp.W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, akq = lane >> 4, jc = lane & 15;
  const int col = grp * SP_N + jc;                 // the spike column of this lane's results
  const int ecol = which == 0 ? ch.a : ch.b + 1;   // coupling column of the unit right-hand side
  const int rcol = which == 0 ? ch.a : ch.b;       // column it sits in
  // the chain: the forward sweep from the loaded end (fcnt steps), the middle column, then
  // the back-substitution towards a (cnt0 steps) and towards b (cnt1 steps)
  const int fcnt = which == 0 ? ch.mid - ch.a : ch.b - ch.mid, cnt0 = ch.mid - ch.a, cnt1 = ch.b - ch.mid;
  const int nsteps = fcnt + 1 + cnt0 + cnt1;
  auto col_at = [&](int t) {
    if (t < fcnt) return which == 0 ? ch.a + t : ch.b - t;
    if (t == fcnt) return ch.mid;
    if (t <= fcnt + cnt0) return ch.mid - (t - fcnt);
    return ch.mid + (t - fcnt - cnt0);
  };
  // the lane's result rows: 16 (wave + NW x) + 4 r + akq = r0 + (16 NW x + 4 r);
  // addresses as a uniform base, the lane's offset and a constant (no clamping: only rows
  // below m are read or written)
  const int r0 = 16 * wave + akq, lo = col * m + r0;
  auto row_of = [&](int x, int r) { return r0 + 16 * NW * x + 4 * r; };
  const double ih2 = -1.0 / (g.h * g.h);
  auto zrow = [&](int x, int r) {   // zn[row] (-1 / h^2), the row factor of the coupling
    const int row = row_of(x, r);
    const C z = row < m ? g.zn[r0 + 16 * NW * x + 4 * r] : make_double2(0.0, 0.0);
    return cscale(z, ih2);
  };
  auto unit = [&](int x, int r) {
    const int row = row_of(x, r);
    return row == col && row < m ? cmul(zrow(x, r), g.ixh[ecol]) : make_double2(0.0, 0.0);
  };
  // right-hand side of the first step: the unit columns (forward), or the middle's
  auto put = [&](int x, int r, C v) {
    const int row = row_of(x, r);
    Bv[row][jc] = row < m ? v : make_double2(0.0, 0.0);
  };
#pragma unroll
  for (int x = 0; x < SW_TW; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) put(x, r, (fcnt > 0 || rcol == ch.mid) ? unit(x, r) : make_double2(0.0, 0.0));
  F64Chain<TPW> A;
  A.init(pp.T, m, lane, wave);
  A.prime(col_at(0));
  for (int t = 0; t < nsteps; ++t) {
    const int i = col_at(t);
    __syncthreads();   // the right-hand side is in Bv
    doublex4 re[SW_TW], im[SW_TW];
    A.product(Bv, i, t + 1 < nsteps ? col_at(t + 1) : i, re, im);
    __syncthreads();   // every wave is done with Bv
    // this step's result (back-substitution: y_i - product, y_i = 0 on the unloaded
    // side), stored; then the next step's right-hand side from it
    const bool back = t > fcnt, side0 = t <= fcnt + cnt0;
    const bool loaded = back && (side0 == (which == 0));
    const int tn = t + 1;
    const bool has_next = tn < nsteps;
    // coupling column of the next step and its kind: 0 forward, 1 middle, 2 back
    int cn = 0, kn = 0;
    if (has_next) {
      const int in = col_at(tn);
      if (tn < fcnt) { kn = 0; cn = which == 0 ? in : in + 1; }
      else if (tn == fcnt) { kn = 1; cn = which == 0 ? ch.mid : ch.mid + 1; }
      else if (tn <= fcnt + cnt0) { kn = 2; cn = in + 1; }
      else { kn = 2; cn = in; }
    }
    const bool restart = has_next && tn == fcnt + cnt0 + 1;   // side b starts again from x_mid
    C *const Oi = Out + (size_t)i * mm;
    const C *const Om = Out + (size_t)ch.mid * mm;
    const C xc = has_next ? g.ixh[cn] : make_double2(0.0, 0.0);
#pragma unroll
    for (int x = 0; x < SW_TW; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(x, r), e = lo + 16 * NW * x + 4 * r;
        const bool ok = row < m && col < m;
        C v = make_double2(re[x][r], im[x][r]);
        if (back) {
          const C y = loaded && ok ? Oi[e] : make_double2(0.0, 0.0);
          v = csub(y, v);
        }
        if (ok) Oi[e] = v;
        if (has_next) {
          if (restart) v = ok ? Om[e] : make_double2(0.0, 0.0);
          const C cj = cmul(zrow(x, r), xc);
          C rhs;
          if (kn == 0) rhs = csub(make_double2(0.0, 0.0), cmul(cj, v));
          else if (kn == 1) rhs = csub(rcol == ch.mid ? unit(x, r) : make_double2(0.0, 0.0), cmul(cj, v));
          else rhs = cmul(cj, v);
          put(x, r, rhs);
        }
      }
  }
}

// FP64 chunk sweeps on the matrix cores (columns up to 144 TPW rows): the steps of
// k_sweep_mfma (item = chunk, side, 16 sources; PH 0 forward, 1 middles, 2
// back-substitution) with the FP64 column product of the spikes (F64Chain, four real
// MFMAs per complex product).  The lanes that hold a step's result also form the next
// step's right-hand side (the coupling is diagonal in the rows), reading b_i or y_i for
// their own entries, so the B operand is the only LDS.
template <int PH, int TPW>
__global__ __launch_bounds__(SweepShape<TPW>::NT, 3) void k_sweep64_mfma(SweepBatch bt) {
  using C = double2;
  constexpr int NW = SweepShape<TPW>::NW;
  extern __shared__ unsigned char smem_raw[];
  C(*Bv)[SP_N + 1] = (C(*)[SP_N + 1])smem_raw;
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int ST = (pp.K + SP_N - 1) / SP_N;
  const int st = local % ST, rest = local / ST;
  const Chunk ch = chunk_of(pp.part, PH == 1 ? rest : rest >> 1);
  const int side = PH == 1 ? 0 : rest & 1;
  const Grid &g = pp.g;
  const int m = g.nz, K = pp.K, s0 = st * SP_N;
  const int cnt = PH == 1 ? 1 : side == 0 ? ch.mid - ch.a : ch.b - ch.mid;
  if (cnt <= 0) return;   // uniform over the workgroup
  auto col_of = [&](int t) {
    return PH == 1 ? ch.mid
                   : PH == 0 ? (side == 0 ? ch.a + t : ch.b - t) : (side == 0 ? ch.mid - 1 - t : ch.mid + 1 + t);
  };
  auto cc_of = [&](int i) { return PH == 0 ? (side == 0 ? i : i + 1) : (side == 0 ? i + 1 : i); };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, akq = lane >> 4, jc = lane & 15;
  const bool sok = s0 + jc < K;
  // the lane's entries: rows 16 (wave + NW x) + 4 r + akq (the f64 D layout) of source
  // s0 + jc, addressed as the lane's base plus a constant
  const int r0 = 16 * wave + akq;
  auto row_of = [&](int x, int r) { return r0 + 16 * NW * x + 4 * r; };
  C *const Xl = (C *)pp.x + (size_t)min(s0 + jc, K - 1) * g.nx * m + r0;
  auto xel = [&](int i, int x, int r) { return Xl + (size_t)i * m + (16 * NW * x + 4 * r); };
  auto ok = [&](int x, int r) { return sok && row_of(x, r) < m; };
  const double ih2 = -1.0 / (g.h * g.h);
  auto zrow = [&](int x, int r) {   // zn[row] (-1 / h^2), the row factor of the coupling
    const C z = row_of(x, r) < m ? g.zn[r0 + 16 * NW * x + 4 * r] : make_double2(0.0, 0.0);
    return cscale(z, ih2);
  };
  auto put = [&](int x, int r, C v) {
    Bv[row_of(x, r)][jc] = ok(x, r) ? v : make_double2(0.0, 0.0);
  };
  auto ld = [&](bool p, const C *a) { return p ? *a : make_double2(0.0, 0.0); };
  // the first step's right-hand side
  {
    const int i0 = col_of(0);
    const C xa = g.ixh[PH == 1 ? ch.mid : cc_of(i0)], xb2 = g.ixh[PH == 1 ? ch.mid + 1 : cc_of(i0)];
    const bool hl = ch.mid > ch.a, hr = ch.mid < ch.b;
#pragma unroll
    for (int x = 0; x < SW_TW; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool o = ok(x, r);
        C rhs;
        if (PH == 0) rhs = ld(o, xel(i0, x, r));   // b at the chunk's end: no coupling inside
        else if (PH == 1) {                        // b_mid - C_mid y_{mid-1} - C_{mid+1} y_{mid+1}
          const C z = zrow(x, r);
          rhs = csub(csub(ld(o, xel(ch.mid, x, r)), cmul(cmul(z, xa), ld(o && hl, xel(ch.mid - 1, x, r)))),
                     cmul(cmul(z, xb2), ld(o && hr, xel(ch.mid + 1, x, r))));
        } else rhs = cmul(cmul(zrow(x, r), xa), ld(o, xel(ch.mid, x, r)));   // C x_mid
        put(x, r, rhs);
      }
  }
  F64Chain<TPW> A;
  A.init((const C *)pp.T, m, lane, wave);
  A.prime(col_of(0));
  for (int t = 0; t < cnt; ++t) {
    const int i = col_of(t);
    __syncthreads();   // the right-hand side is in Bv
    doublex4 re[SW_TW], im[SW_TW];
    A.product(Bv, i, t + 1 < cnt ? col_of(t + 1) : i, re, im);
    __syncthreads();   // every wave is done with Bv
    const bool more = t + 1 < cnt;
    const int in = more ? col_of(t + 1) : i;
    const C xc = g.ixh[cc_of(in)];
#pragma unroll
    for (int x = 0; x < SW_TW; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool o = ok(x, r);
        C v = make_double2(re[x][r], im[x][r]);
        if (PH == 2) v = csub(ld(o, xel(i, x, r)), v);   // x_i = y_i - T_i C x_prev
        if (o) *xel(i, x, r) = v;
        if (more) {
          const C cj = cmul(zrow(x, r), xc);
          put(x, r, PH == 0 ? csub(ld(o, xel(in, x, r)), cmul(cj, v)) : cmul(cj, v));
        }
      }
  }
}

template <typename R, int NS, int PH>
__global__ __launch_bounds__((SolveThreads<R, NS>::N)) void k_solve(SweepBatch bt) {
  extern __shared__ unsigned char smem[];
  const int item = item_of_block(bt.xs);
  if (item < 0) return;
  const int q = find_problem(bt.first, bt.n, item);
  const SweepProblem &pp = bt.p[q];
  const int local = item - bt.first[q];
  const int G = (pp.K + NS - 1) / NS;
  const int grp = local % G, rest = local / G;
  const cplx<R> *T = (const cplx<R> *)pp.T;
  if (PH == 0)
    fwd_body<R, NS>(pp.g, pp.K, chunk_of(pp.part, rest >> 1), T, pp.x, grp, rest & 1, smem);
  else if (PH == 1)
    mid_body<R, NS>(pp.g, pp.K, chunk_of(pp.part, rest), T, pp.x, grp, smem);
  else if (PH == 2)
    bwd_body<R, NS>(pp.g, pp.K, chunk_of(pp.part, rest >> 1), T, pp.x, grp, rest & 1, smem);
  else
    red_rhs_body<R, NS>(pp.g, pp.K, separator(pp.part, rest + 1), pp.x, grp);
}

// Row-major fields [K][nz][nx] (IO type) to the column-major compute copy [K][nx][nz]
// and back, through 32 x 32 LDS tiles (coalesced on both sides); ADJ conjugates.
// grid (ceil(nx/32), ceil(nz/32), K), block (32, 8).
template <typename R, typename IO, bool ADJ>
__global__ __launch_bounds__(256) void k_to_colmajor(Grid g, const IO *__restrict__ in, cplx<R> *__restrict__ out) {
  __shared__ cplx<R> tile[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32, k = blockIdx.z;
  const size_t Nu = (size_t)g.nx * g.nz;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + threadIdx.x;
    if (j < g.nz && i < g.nx) {
      const IO v = in[k * Nu + (size_t)j * g.nx + i];
      cplx<R> c = mk<R>((R)v.x, (R)v.y);
      tile[r][threadIdx.x] = ADJ ? cconj(c) : c;
    }
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + threadIdx.x;
    if (i < g.nx && j < g.nz) out[k * Nu + (size_t)i * g.nz + j] = tile[threadIdx.x][r];
  }
}
template <typename R, typename IO, bool ADJ>
__global__ __launch_bounds__(256) void k_from_colmajor(Grid g, const cplx<R> *__restrict__ in, IO *__restrict__ out) {
  __shared__ cplx<R> tile[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32, k = blockIdx.z;
  const size_t Nu = (size_t)g.nx * g.nz;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + threadIdx.x;
    if (i < g.nx && j < g.nz) tile[threadIdx.x][r] = in[k * Nu + (size_t)i * g.nz + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + threadIdx.x;
    if (j < g.nz && i < g.nx) {
      cplx<R> c = tile[r][threadIdx.x];
      if (ADJ) c = cconj(c);
      IO v;
      v.x = c.x;
      v.y = c.y;
      out[k * Nu + (size_t)j * g.nx + i] = v;
    }
  }
}

// block shape of the sweeps: x covers the rows, y splits each dot product (at most
// `threads` threads)
inline dim3 sweep_block(int m, int threads = 512) {
  int rj = ((m + 63) / 64) * 64;
  int gy = threads / rj;
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

// ---------------------------------------------------------------------------
// the XCD ranges of a launch: items [first[q], first[q+1]) of problem q cost cost[q]
// each; the 8 ranges are cut at equal cumulative cost.  Returns the grid size.
// ---------------------------------------------------------------------------
static unsigned xcd_split(const int *first, int n, const double *cost, int *xs) {
  double total = 0.0;
  for (int q = 0; q < n; ++q) total += (first[q + 1] - first[q]) * cost[q];
  xs[0] = 0;
  xs[8] = first[n];
  for (int x = 1; x < 8; ++x) {
    const double target = total * x / 8.0;
    int idx = first[n];
    double cum = 0.0;
    for (int q = 0; q < n; ++q) {
      const double c = (first[q + 1] - first[q]) * cost[q];
      if (c > 0.0 && cum + c >= target) {
        idx = first[q] + (int)std::ceil((target - cum) / cost[q]);
        idx = std::min(std::max(idx, first[q]), first[q + 1]);
        break;
      }
      cum += c;
    }
    xs[x] = std::max(xs[x - 1], std::min(idx, first[n]));
  }
  int most = 0;
  for (int x = 0; x < 8; ++x) most = std::max(most, xs[x + 1] - xs[x]);
  return 8u * (unsigned)most;
}

// ---------------------------------------------------------------------------
// partition of the columns
// ---------------------------------------------------------------------------
int blu_auto_chunks(int nx, int nz, int K) {
  (void)nz; (void)K;
  if (nx < 32) return 1;
  // the separators cost log2(P) levels, so chunks of ~sqrt(nx) / 1.6 columns
  int P = (int)std::lround(1.6 * std::sqrt((double)nx));
  return std::max(1, std::min({P, KF_MAX_CHUNKS, (nx + 1) / 2}));
}

kf_status blu_set_shape(kf_problem *p, int chunks, int ns) {
  if (chunks == 0) chunks = blu_auto_chunks(p->nx, p->nz, p->K);
  if (chunks < 1 || chunks > KF_MAX_CHUNKS || 2 * chunks - 1 > p->nx) {
    set_error("chunks must be in 1 .. min(64, (nx + 1) / 2)");
    return KF_EINVAL;
  }
  if (ns == 0) ns = 1;
  if (ns != 1 && ns != 2 && ns != 4 && ns != 8) {
    set_error("sources per workgroup must be 1, 2, 4 or 8");
    return KF_EINVAL;
  }
  p->ns = ns;
  if (chunks == p->P && !p->part.empty()) return KF_OK;
  const int m = p->nz;
  const size_t mm = (size_t)m * m;
  // P chunks around P - 1 separators, interior lengths as even as possible
  std::vector<int> part(3 * chunks);
  const int n_int = p->nx - (chunks - 1), base = n_int / chunks, extra = n_int % chunks;
  int a = 0;
  for (int c = 0; c < chunks; ++c) {
    const int L = base + (c < extra ? 1 : 0);
    part[3 * c] = a;
    part[3 * c + 1] = a + L - 1;
    part[3 * c + 2] = a + L / 2;
    a += L + 1;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  HIP_TRY(hipMemcpy(p->d_part, part.data(), sizeof(int) * part.size(), hipMemcpyHostToDevice));
  const size_t slots = 2 * (size_t)chunks;
  if (slots > p->fac_slots) {
    if (p->fac_work) HIP_TRY(hipFree(p->fac_work));
    p->fac_work = nullptr;
    p->fac_slots = 0;
    HIP_TRY(kf_malloc((void **)&p->fac_work, sizeof(double2) * slots * (mm + (size_t)NB_MAX * m)));
    p->fac_slots = slots;
  }
  if (chunks > 1 && !p->V64) {
    const size_t n = (size_t)p->nx * mm;
    HIP_TRY(kf_malloc((void **)&p->V64, sizeof(double2) * n));
    HIP_TRY(kf_malloc((void **)&p->W64, sizeof(double2) * n));
    HIP_TRY(kf_malloc((void **)&p->V32, sizeof(float2) * n));
    HIP_TRY(kf_malloc((void **)&p->W32, sizeof(float2) * n));
  }
  // the separators' reduction blocks, sized by the separator count
  for (void *q : {(void *)p->CRL64, (void *)p->CR64, (void *)p->CR32, (void *)p->sep32, (void *)p->corr_e,
                  (void *)p->cr_part})
    if (q) HIP_TRY(hipFree(q));
  p->CRL64 = p->CR64 = nullptr;
  p->CR32 = p->sep32 = nullptr;
  p->corr_e = nullptr;
  p->cr_part = nullptr;
  if (chunks > 1) {
    const size_t nsep = chunks - 1;
    HIP_TRY(kf_malloc((void **)&p->CRL64, sizeof(double2) * nsep * 4 * mm));
    HIP_TRY(kf_malloc((void **)&p->CR64, sizeof(double2) * nsep * CR_LV * 2 * mm));
    HIP_TRY(kf_malloc((void **)&p->CR32, sizeof(float2) * nsep * CR_LV * 2 * mm));
    HIP_TRY(kf_malloc((void **)&p->sep32, sizeof(float2) * nsep * p->K * m));
    HIP_TRY(kf_malloc((void **)&p->corr_e, sizeof(int) * chunks * p->K));
    // the terms' partials of a reduction level: complex64, at most one tile per
    // (separator, row tile, source tile); FP64, one m-vector per (separator, source),
    // source groups padded
    const size_t crt = nsep * ((m + CRM_R - 1) / CRM_R) * ((p->K + CRM_S - 1) / CRM_S);
    const size_t b32 = sizeof(float2) * crt * 3 * CRM_S * CRM_R;
    const size_t b64 = sizeof(double2) * nsep * (p->K + 8) * 3 * (size_t)m;
    HIP_TRY(kf_malloc((void **)&p->cr_part, std::max(b32, b64)));
    if (!p->vwh) {   // independent of the partition
      p->vw_k2 = 2 * ((m + 31) / 32 * 32);
      HIP_TRY(kf_malloc((void **)&p->vwh, sizeof(uint16_t) * 4 * (size_t)p->nx * m * p->vw_k2));
      HIP_TRY(kf_malloc((void **)&p->vwe, sizeof(int) * p->nx));
    }
  }
  p->part = part;
  p->P = chunks;
  int lmax = 0;
  for (int c = 0; c < chunks; ++c) lmax = std::max(lmax, part[3 * c + 1] - part[3 * c] + 1);
  p->lmax = lmax;
  p->have_T64 = p->have_T32 = false;
  return KF_OK;
}

// ---------------------------------------------------------------------------
// factorisation of a batch of problems (a single problem is a batch of one)
// ---------------------------------------------------------------------------
namespace {
// every matrix of the job range inverted: GJ_NB-column panels, one launch each, then
// the transposed store
kf_status gj_invert(const GjJob *dj, int cnt, int m_max, hipStream_t s) {
  if (cnt == 0) return KF_OK;
  const int npan = (m_max + GJ_NB - 1) / GJ_NB, nt = 64 * ((m_max + 63) / 64);
  for (int t = 0; t <= npan; ++t) {
    hipLaunchKernelGGL((k_gj_step<GJ_NB>), dim3(npan, cnt), dim3(nt), 0, s, dj, t);
    LAUNCH_CHECK();
  }
  const int t32 = (m_max + 31) / 32;
  hipLaunchKernelGGL((k_gj_store<GJ_NB>), dim3(t32 * t32, cnt), dim3(256), 0, s, dj);
  LAUNCH_CHECK();
  return KF_OK;
}

kf_status factor64_launch(const std::vector<kf_problem *> &ps, hipStream_t s, int m_max) {
  if (m_max > 512) { set_error("column height above 512"); return KF_EINVAL; }
  FactorBatch bt{};
  bt.n = (int)ps.size();
  for (int q = 0; q < bt.n; ++q) {
    kf_problem *p = ps[q];
    bt.p[q] = FactorProblem{p->grid(), p->P, p->d_part, p->T64, p->V64, p->W64, p->fac_work};
  }
  auto slot = [](kf_problem *p, int i) { return p->fac_work + (size_t)i * ((size_t)p->nz * p->nz + (size_t)NB_MAX * p->nz); };
  auto tblk = [](kf_problem *p, int col) { return p->T64 + (size_t)col * p->nz * p->nz; };
  // 1. job tables of the chunks' twisted factorisations: step st of every (chunk,
  //    side) chain that has one (side 0 walks a..mid-1, side 1 b..mid+1), then the
  //    middle columns.  A step is a Schur complement and an inversion per chain.
  std::vector<SchurJob> sjobs;
  std::vector<GjJob> gjobs;
  struct ChainStep { int off, cnt; };
  std::vector<ChainStep> chain;
  int maxcnt = 0;
  for (kf_problem *p : ps)
    for (int c = 0; c < p->P; ++c)
      maxcnt = std::max(maxcnt, std::max(p->part[3 * c + 2] - p->part[3 * c], p->part[3 * c + 1] - p->part[3 * c + 2]));
  for (int st = 0; st <= maxcnt; ++st) {
    ChainStep cs{(int)sjobs.size(), 0};
    for (int q = 0; q < bt.n; ++q) {
      kf_problem *p = ps[q];
      const int m = p->nz;
      for (int c = 0; c < p->P; ++c) {
        const int a = p->part[3 * c], b = p->part[3 * c + 1], mid = p->part[3 * c + 2];
        if (st == maxcnt) {   // the middle columns
          const bool hl = mid > a, hr = mid < b;
          double2 *S = slot(p, 2 * c);
          sjobs.push_back(SchurJob{q, mid, hl ? mid : -1, hr ? mid + 1 : -1, hl ? tblk(p, mid - 1) : nullptr,
                                   hr ? tblk(p, mid + 1) : nullptr, S});
          gjobs.push_back(GjJob{m, S, tblk(p, mid)});
          cs.cnt++;
          continue;
        }
        for (int side = 0; side < 2; ++side) {
          const int cnt = side == 0 ? mid - a : b - mid;
          if (st >= cnt) continue;
          const int i = side == 0 ? a + st : b - st;
          const bool has = st > 0;
          const int prev = side == 0 ? i - 1 : i + 1, cc = side == 0 ? i : i + 1;
          double2 *S = slot(p, 2 * c + side);
          sjobs.push_back(SchurJob{q, i, has ? cc : -1, -1, has ? tblk(p, prev) : nullptr, nullptr, S});
          gjobs.push_back(GjJob{m, S, tblk(p, i)});
          cs.cnt++;
        }
      }
    }
    chain.push_back(cs);
  }
  // 2. job tables of the separators' reduction (all problems, level by level)
  int ntot = 0, top_max = -1;
  int sep_first[KF_BATCH_MAX];
  for (int q = 0; q < bt.n; ++q) {
    sep_first[q] = ntot;
    const int nsep = ps[q]->P - 1;
    ntot += nsep;
    if (nsep > 0) top_max = std::max(top_max, cr_top(nsep));
  }
  std::vector<CrJob> jobs;
  struct Step { int kind, off, cnt; };   // kind 0 copy, 1 invert (GjJob range), 2 gemm
  std::vector<Step> steps;
  {
    auto sep = [](kf_problem *p, int j) { return p->part[3 * (j - 1) + 1] + 1; };
    auto blk = [](kf_problem *p, double2 *base, int col) { return base + (size_t)col * p->nz * p->nz; };
    auto lu = [](kf_problem *p, int j, int w) { return p->CRL64 + ((size_t)(j - 1) * 4 + w) * p->nz * p->nz; };
    auto crb = [](kf_problem *p, int k, int lv, int w) {
      return p->CR64 + (((size_t)(k - 1) * CR_LV + lv) * 2 + w) * p->nz * p->nz;
    };
    auto begin = [&](int kind) { steps.push_back(Step{kind, (int)jobs.size(), 0}); };
    auto add = [&](const CrJob &j) { jobs.push_back(j); steps.back().cnt++; };
    for (int lv = 0; lv <= top_max; ++lv) {
      // A: invert the separators eliminated at this level (and each problem's root at its top)
      std::vector<std::pair<kf_problem *, int>> inv;
      for (kf_problem *p : ps) {
        const int n = p->P - 1;
        if (n < 1) continue;
        const int top = cr_top(n), st = 1 << lv;
        if (lv < top)
          for (int j = st; j <= n; j += 2 * st) inv.push_back({p, j});
        else if (lv == top)
          inv.push_back({p, 1 << top});
      }
      if (inv.empty()) continue;
      std::map<kf_problem *, int> used;
      begin(0);
      for (auto &e : inv) {
        const int i = used[e.first]++;
        add(CrJob{e.first->nz, 1.0, blk(e.first, e.first->T64, sep(e.first, e.second)), nullptr, nullptr, slot(e.first, i)});
      }
      used.clear();
      steps.push_back(Step{1, (int)gjobs.size(), 0});
      for (auto &e : inv) {
        const int i = used[e.first]++;
        gjobs.push_back(GjJob{e.first->nz, slot(e.first, i), blk(e.first, e.first->T64, sep(e.first, e.second))});
        steps.back().cnt++;
      }
      // B: F_j = Binv_j L_j, G_j = Binv_j U_j
      begin(2);
      for (kf_problem *p : ps) {
        const int n = p->P - 1;
        if (n < 1 || lv >= cr_top(n)) continue;
        const int st = 1 << lv;
        for (int j = st; j <= n; j += 2 * st) {
          const int s_ = sep(p, j);
          if (j - st >= 1) add(CrJob{p->nz, 1.0, blk(p, p->T64, s_), lu(p, j, 0), nullptr, blk(p, p->V64, s_)});
          if (j + st <= n) add(CrJob{p->nz, 1.0, blk(p, p->T64, s_), lu(p, j, 1), nullptr, blk(p, p->W64, s_)});
        }
      }
      // C: B_k -= L_k G_j1, ML, MU, and the next level's L, U (staging)
      begin(2);
      for (kf_problem *p : ps) {
        const int n = p->P - 1;
        if (n < 1 || lv >= cr_top(n)) continue;
        const int st = 1 << lv;
        for (int k = 2 * st; k <= n; k += 2 * st) {
          const int sk = sep(p, k), s1 = sep(p, k - st), j2 = k + st;
          add(CrJob{p->nz, -1.0, lu(p, k, 0), blk(p, p->W64, s1), blk(p, p->T64, sk), blk(p, p->T64, sk)});
          add(CrJob{p->nz, 1.0, lu(p, k, 0), blk(p, p->T64, s1), nullptr, crb(p, k, lv, 0)});
          if (k - 2 * st >= 1) add(CrJob{p->nz, -1.0, lu(p, k, 0), blk(p, p->V64, s1), nullptr, lu(p, k, 2)});
          if (j2 <= n) {
            const int s2 = sep(p, j2);
            add(CrJob{p->nz, 1.0, lu(p, k, 1), blk(p, p->T64, s2), nullptr, crb(p, k, lv, 1)});
            if (j2 + st <= n) add(CrJob{p->nz, -1.0, lu(p, k, 1), blk(p, p->W64, s2), nullptr, lu(p, k, 3)});
          }
        }
      }
      // D: B_k -= U_k F_j2
      begin(2);
      for (kf_problem *p : ps) {
        const int n = p->P - 1;
        if (n < 1 || lv >= cr_top(n)) continue;
        const int st = 1 << lv;
        for (int k = 2 * st; k + st <= n; k += 2 * st) {
          const int sk = sep(p, k);
          add(CrJob{p->nz, -1.0, lu(p, k, 1), blk(p, p->V64, sep(p, k + st)), blk(p, p->T64, sk), blk(p, p->T64, sk)});
        }
      }
      // E: the next level's L_k, U_k (zero where the neighbour has none)
      begin(0);
      for (kf_problem *p : ps) {
        const int n = p->P - 1;
        if (n < 1 || lv >= cr_top(n)) continue;
        const int st = 1 << lv;
        for (int k = 2 * st; k <= n; k += 2 * st) {
          add(CrJob{p->nz, 0.0, k - 2 * st >= 1 ? lu(p, k, 2) : nullptr, nullptr, nullptr, lu(p, k, 0)});
          add(CrJob{p->nz, 0.0, (k + st <= n && k + 2 * st <= n) ? lu(p, k, 3) : nullptr, nullptr, nullptr, lu(p, k, 1)});
        }
      }
    }
  }
  // 3. one upload of every table (the previous factorisation's launches must be done
  //    with the buffer first: it lives in the first problem)
  const size_t sz_s = sizeof(SchurJob) * sjobs.size(), sz_g = sizeof(GjJob) * gjobs.size();
  const size_t off_g = (sz_s + 255) & ~(size_t)255, off_c = (off_g + sz_g + 255) & ~(size_t)255;
  const size_t bytes = off_c + sizeof(CrJob) * jobs.size();
  kf_problem *p0 = ps[0];
  HIP_TRY(hipStreamSynchronize(s));
  if (bytes > p0->fac_jobs_cap) {
    if (p0->fac_jobs) HIP_TRY(hipFree(p0->fac_jobs));
    p0->fac_jobs = nullptr;
    p0->fac_jobs_cap = 0;
    HIP_TRY(kf_malloc(&p0->fac_jobs, bytes));
    p0->fac_jobs_cap = bytes;
  }
  std::vector<unsigned char> host(bytes, 0);
  if (sz_s) std::memcpy(host.data(), sjobs.data(), sz_s);
  if (sz_g) std::memcpy(host.data() + off_g, gjobs.data(), sz_g);
  if (!jobs.empty()) std::memcpy(host.data() + off_c, jobs.data(), sizeof(CrJob) * jobs.size());
  HIP_TRY(hipMemcpy(p0->fac_jobs, host.data(), bytes, hipMemcpyHostToDevice));
  const SchurJob *dsj = (const SchurJob *)p0->fac_jobs;
  const GjJob *dgj = (const GjJob *)((unsigned char *)p0->fac_jobs + off_g);
  const CrJob *dj = (const CrJob *)((unsigned char *)p0->fac_jobs + off_c);
  // 4. the chunks: Schur complement and inversion, chain step by chain step
  const int t32 = (m_max + 31) / 32;
  for (const ChainStep &cs : chain) {
    if (cs.cnt == 0) continue;
    hipLaunchKernelGGL(k_schur, dim3(t32 * t32, cs.cnt), dim3(256), 0, s, bt, dsj + cs.off);
    LAUNCH_CHECK();
    kf_status st = gj_invert(dgj + cs.off, cs.cnt, m_max, s);
    if (st != KF_OK) return st;
  }
  // 5. spikes
  double cost[KF_BATCH_MAX];
  int tot = 0;
  for (int q = 0; q < bt.n; ++q) {
    const double m = ps[q]->nz, L = (double)ps[q]->nx / ps[q]->P;
    bt.first[q] = tot;
    tot += 2 * (ps[q]->P - 1) * ((ps[q]->nz + SP_N - 1) / SP_N);
    cost[q] = m * m * 1.5 * L;
  }
  bt.first[bt.n] = bt.total = tot;
  if (tot == 0) return KF_OK;   // one chunk: no separators
  const unsigned grid_sp = xcd_split(bt.first, bt.n, cost, bt.xs);
  // columns up to 288 rows on the matrix cores, taller ones on the vector units
  if (m_max <= SweepShape<1>::M) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_spikes_mfma<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)f64_chain_lds<1>()));
    hipLaunchKernelGGL(k_spikes_mfma<1>, dim3(grid_sp), dim3(SweepShape<1>::NT), f64_chain_lds<1>(), s, bt);
  } else if (m_max <= SweepShape<2>::M) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_spikes_mfma<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)f64_chain_lds<2>()));
    hipLaunchKernelGGL(k_spikes_mfma<2>, dim3(grid_sp), dim3(SweepShape<2>::NT), f64_chain_lds<2>(), s, bt);
  } else {
    const size_t smem_sp = (size_t)m_max * SP_N * sizeof(double2);
    HIP_TRY(hipFuncSetAttribute((const void *)k_spikes, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_sp));
    hipLaunchKernelGGL(k_spikes, dim3(grid_sp), dim3(2 * spike_pairs_padded(m_max)), smem_sp, s, bt);
  }
  LAUNCH_CHECK();
  // 6. the separators' system by block cyclic reduction
  if (ntot == 0) return KF_OK;
  for (int q = 0; q < bt.n; ++q) bt.first[q] = sep_first[q];
  bt.first[bt.n] = bt.total = ntot;
  for (int q = 0; q < bt.n; ++q) bt.p[q].lu = ps[q]->CRL64;
  hipLaunchKernelGGL(k_cr_setup, dim3(std::min(256, (m_max * m_max + 255) / 256), ntot), dim3(256), 0, s, bt);
  LAUNCH_CHECK();
  const int tiles = t32 * t32;
  const int cblocks = std::min(64, (m_max * m_max + 255) / 256);
  for (const Step &stp : steps) {
    if (stp.cnt == 0) continue;
    if (stp.kind == 0) hipLaunchKernelGGL(k_cr_copy, dim3(cblocks, stp.cnt), dim3(256), 0, s, dj + stp.off);
    else if (stp.kind == 1) {
      kf_status st = gj_invert(dgj + stp.off, stp.cnt, m_max, s);
      if (st != KF_OK) return st;
    } else hipLaunchKernelGGL(k_cr_gemm, dim3(tiles, stp.cnt), dim3(256), 0, s, dj + stp.off);
    LAUNCH_CHECK();
  }
  return KF_OK;
}
}  // namespace

kf_status blu_factor_batch(const std::vector<kf_problem *> &all, int which, hipStream_t s) {
  std::vector<kf_problem *> ps;
  int m_max = 0;
  for (kf_problem *p : all)
    if ((which & 3) && !p->have_T64) { ps.push_back(p); m_max = std::max(m_max, p->nz); }
  if ((int)ps.size() > KF_BATCH_MAX) { set_error("batch too large"); return KF_EINVAL; }
  if (!ps.empty()) {
    kf_status st = factor64_launch(ps, s, m_max);
    if (st != KF_OK) return st;
    for (kf_problem *p : ps) p->have_T64 = true;
  }
  if (which & 2)
    for (kf_problem *p : all)
      if (!p->have_T32) {
        const int64_t n = (int64_t)p->nx * p->nz * p->nz;
        kf_status st = launch_copy_c128_to_c64(p, n, p->T64, p->T32);
        if (st == KF_OK && p->P > 1) st = launch_copy_c128_to_c64(p, n, p->V64, p->V32);
        if (st == KF_OK && p->P > 1) st = launch_copy_c128_to_c64(p, n, p->W64, p->W32);
        if (st == KF_OK && p->P > 1) {   // the spikes as scaled FP16 pairs for the interior correction
          hipLaunchKernelGGL(k_spike_exponents, dim3(p->nx), dim3(256), 0, p->stream, p->grid(), p->P, p->d_part,
                             p->V32, p->W32, p->vwe);
          LAUNCH_CHECK();
          const int jt = (p->nz + 31) / 32, kt = p->vw_k2 / 32;
          hipLaunchKernelGGL(k_spike_split, dim3(jt * kt, p->nx), dim3(256), 0, p->stream, p->grid(), p->P,
                             p->d_part, p->V32, p->W32, p->vwe, p->vw_k2, p->vwh);
          LAUNCH_CHECK();
        }
        if (st == KF_OK && p->P > 1)
          st = launch_copy_c128_to_c64(p, (int64_t)(p->P - 1) * CR_LV * 2 * p->nz * p->nz, p->CR64, p->CR32);
        if (st != KF_OK) return st;
        p->have_T32 = true;
      }
  return KF_OK;
}

kf_status blu_factor(kf_problem *p, int which) {
  if (which & 3) {
    if (!p->have_T64) {
      ProfScope ps(p, PROF_FACTOR);
      kf_status st = blu_factor_batch({p}, 1, p->stream);
      if (st != KF_OK) return st;
    }
    if ((which & 2) && !p->have_T32) return blu_factor_batch({p}, 2, p->stream);
  }
  return KF_OK;
}

// ---------------------------------------------------------------------------
// solves of a batch of problems: the column-major copy, six phases (one launch
// each, covering every problem), and the copy back
// ---------------------------------------------------------------------------
namespace {
template <typename R, int NS>
kf_status solve_phases(const std::vector<kf_problem *> &ps, hipStream_t s, kf_problem *prof) {
  const bool fp32 = sizeof(R) == sizeof(float);
  SweepBatch bt{};
  bt.n = (int)ps.size();
  int m_max = 0;
  for (int q = 0; q < bt.n; ++q) {
    kf_problem *p = ps[q];
    m_max = std::max(m_max, p->nz);
    bt.p[q] = SweepProblem{p->grid(), p->K, p->P, p->lmax, p->d_part,
                           fp32 ? (const void *)p->T32 : (const void *)p->T64,
                           fp32 ? (const void *)p->V32 : (const void *)p->V64,
                           fp32 ? (const void *)p->W32 : (const void *)p->W64,
                           fp32 ? (const void *)p->CR32 : (const void *)p->CR64,
                           fp32 ? (void *)p->sol32 : (void *)p->sol64, (void *)p->sep32, p->vwh, p->vwe,
                           p->corr_e, p->vw_k2, p->cr_part};
  }
  const dim3 blk = sweep_block(m_max, SolveThreads<R, NS>::N);
  const size_t smem = (2 + (blk.y - 1)) * NS * (size_t)m_max * sizeof(cplx<R>);
  if (smem > 65536) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_solve<R, NS, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    HIP_TRY(hipFuncSetAttribute((const void *)k_solve<R, NS, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    HIP_TRY(hipFuncSetAttribute((const void *)k_solve<R, NS, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  }
  constexpr int NSC = CrSources<R, NS>::N;
  // the reduction's levels: flat workgroups (row, column group), see cr_terms
  const dim3 blkc(SolveThreadsCR<R, NSC>::N);
  const size_t smemc = (3 * (size_t)m_max + SolveThreadsCR<R, NSC>::N) * NSC * sizeof(cplx<R>);
  if (smemc > 65536) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_cr_solve<R, NSC, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smemc));
    HIP_TRY(hipFuncSetAttribute((const void *)k_cr_solve<R, NSC, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smemc));
    HIP_TRY(hipFuncSetAttribute((const void *)k_cr_solve<R, NSC, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smemc));
  }
  // launch order: 0 forward sweeps, 1 middle columns, 2 back-substitution, 3 separator
  // right-hand sides, the separators' reduction (forward levels, root, back levels),
  // then 5 the interior correction
  int top_max = -1;
  for (kf_problem *p : ps)
    if (p->P > 1) top_max = std::max(top_max, cr_top(p->P - 1));
  std::vector<std::pair<int, int>> seq;   // (phase, level); phase 4: 0 fwd, 1 root, 2 bwd in .second / 16
  for (int ph = 0; ph < 4; ++ph) seq.push_back({ph, 0});
  for (int lv = 0; lv < top_max; ++lv) seq.push_back({4, lv});
  if (fp32 && top_max >= 0) seq.push_back({6, 0});   // stage g at the separators (matrix-core levels)
  if (top_max >= 0) seq.push_back({4, 16});
  for (int lv = top_max - 1; lv >= 0; --lv) seq.push_back({4, 32 + lv});
  seq.push_back({5, 0});
  static const int ids[7] = {-1, PROF_MID, -1, PROF_REDRHS, PROF_CHAIN, PROF_CORRECT, PROF_CHAIN};
  // chunk sweeps and middles on the matrix cores (FP32 or FP64) where the columns fit the
  // kernels (up to 144 rows: 3 waves, up to 288: 6 waves of three row tiles); in a batch
  // each problem takes its own kind: sweep group 0 (144), 1 (288), 2 (vector units)
  auto sweep_group = [&](const kf_problem *p) {
    return p->nz <= SweepShape<1>::M ? 0 : p->nz <= SweepShape<2>::M ? 1 : 2;
  };
  if (fp32) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<0, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<0, 1>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<2, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<2, 1>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<0, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<0, 2>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<2, 2>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<1, 1>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep_mfma<1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sweep_mfma_lds<1, 2>()));
  } else {
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep64_mfma<0, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)f64_chain_lds<2>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep64_mfma<1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)f64_chain_lds<2>()));
    HIP_TRY(hipFuncSetAttribute((const void *)k_sweep64_mfma<2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)f64_chain_lds<2>()));
  }
  // a matrix-core sweep phase for sweep group sg < 2
  auto mfma_sweep = [&](auto phc, int sg, unsigned grid) {
    constexpr int PH = decltype(phc)::value;
    if (fp32) {
      if (sg == 1) hipLaunchKernelGGL((k_sweep_mfma<PH, 2>), dim3(grid), dim3(SweepShape<2>::NT), (sweep_mfma_lds<PH, 2>()), s, bt);
      else hipLaunchKernelGGL((k_sweep_mfma<PH, 1>), dim3(grid), dim3(SweepShape<1>::NT), (sweep_mfma_lds<PH, 1>()), s, bt);
    } else {
      if (sg == 1) hipLaunchKernelGGL((k_sweep64_mfma<PH, 2>), dim3(grid), dim3(SweepShape<2>::NT), f64_chain_lds<2>(), s, bt);
      else hipLaunchKernelGGL((k_sweep64_mfma<PH, 1>), dim3(grid), dim3(SweepShape<1>::NT), f64_chain_lds<1>(), s, bt);
    }
  };
  for (const auto &e : seq) {
    const int ph = e.first, kind = e.second >> 4, lv = e.second & 15;
    // phases 0-2 run once per sweep group (problems of other groups get no items)
    for (int sg = (ph <= 2 ? 0 : -1); sg <= (ph <= 2 ? 2 : -1); ++sg) {
      int tot = 0;
      double cost[KF_BATCH_MAX];
      for (int q = 0; q < bt.n; ++q) {
        const kf_problem *p = ps[q];
        const int G = (p->K + (ph == 4 ? NSC : NS) - 1) / (ph == 4 ? NSC : NS), n = p->P - 1;
        const int STs = (p->K + SW_S - 1) / SW_S;
        const double m = p->nz, L = (double)p->nx / p->P;
        // a matrix-core sweep step costs its fixed 144 TPW-row tile whatever m is
        const double mt = ph <= 2 && sg < 2 ? 144.0 * (sg + 1) : m;
        cost[q] = ph == 0 || ph == 2 ? mt * mt * 0.5 * L : ph == 5 || ph == 6 ? m : mt * mt;
        // matrix-core reduction levels: (separator, row tile, source tile, term) items
        const int CT = ((p->nz + CRM_R - 1) / CRM_R) * ((p->K + CRM_S - 1) / CRM_S);
        const int GL = fp32 ? CT * cr_split(kind) : G * cr_split64(kind);
        bt.first[q] = tot;
        int items = 0;
        if (ph <= 2 && sweep_group(p) != sg) items = 0;
        else if (ph == 0 || ph == 2) items = 2 * p->P * (sg < 2 ? STs : G);
        else if (ph == 1) items = p->P * (sg < 2 ? STs : G);
        else if (ph == 3) items = n * G;
        else if (ph == 4) {
          if (n >= 1) {
            const int top = cr_top(n);
            if (kind == 0 && lv < top) items = (n >> (lv + 1)) * GL;
            else if (kind == 1) items = GL;   // the root, a launch of its own
            else if (kind == 2 && lv < top) items = (((n >> lv) + 1) / 2) * GL;
          }
        } else if (ph == 6) {
          items = n * p->K;
        } else if (p->P > 1) {
          items = p->P * (fp32 ? ((p->lmax * p->nz + CH_R - 1) / CH_R) * ((p->K + CH_S - 1) / CH_S)
                               : ((p->lmax * p->nz + CG_R - 1) / CG_R) * ((p->K + CG_S - 1) / CG_S));
        }
        tot += items;
      }
      bt.first[bt.n] = bt.total = tot;
      bt.level = lv;
      if (tot == 0) continue;
      const unsigned grid = xcd_split(bt.first, bt.n, cost, bt.xs);
      // algorithmic bytes of a reduction level (single problem): its m x m blocks once,
      // and per source the separators' vectors it reads and writes (edge separators,
      // which have one term less, are counted with all terms)
      double work = 0.0;
      if (ph == 4 && prof && prof->P > 1) {
        const int n = prof->P - 1, top = cr_top(n);
        const double m = prof->nz, esz = 2.0 * sizeof(R);
        int cnt = 0, terms = 0;
        if (kind == 0 && lv < top) { cnt = n >> (lv + 1); terms = 2 * cnt; }
        else if (kind == 1) { cnt = 1; terms = 1; }
        else if (kind == 2 && lv < top) { cnt = ((n >> lv) + 1) / 2; terms = 3 * cnt; }
        work = esz * (terms * m * m + (double)(terms + cnt) * prof->K * m);
      }
      ProfScope pf(prof, ph == 0 ? (fp32 ? PROF_FWD32 : PROF_FWD64) : ph == 2 ? (fp32 ? PROF_BWD32 : PROF_BWD64) : ids[ph],
                   work);
      switch (ph) {
        case 0:
          if (sg < 2) mfma_sweep(std::integral_constant<int, 0>(), sg, grid);
          else hipLaunchKernelGGL((k_solve<R, NS, 0>), dim3(grid), blk, smem, s, bt);
          break;
        case 1:
          if (sg < 2) mfma_sweep(std::integral_constant<int, 1>(), sg, grid);
          else hipLaunchKernelGGL((k_solve<R, NS, 1>), dim3(grid), blk, smem, s, bt);
          break;
        case 2:
          if (sg < 2) mfma_sweep(std::integral_constant<int, 2>(), sg, grid);
          else hipLaunchKernelGGL((k_solve<R, NS, 2>), dim3(grid), blk, smem, s, bt);
          break;
        case 3: hipLaunchKernelGGL((k_solve<R, NS, 3>), dim3(grid), blk, smem, s, bt); break;
        case 4:
          if (fp32) {
            if (kind == 0) hipLaunchKernelGGL(k_cr_mfma<0>, dim3(grid), dim3(256), 0, s, bt);
            else if (kind == 1) hipLaunchKernelGGL(k_cr_mfma<1>, dim3(grid), dim3(256), 0, s, bt);
            else hipLaunchKernelGGL(k_cr_mfma<2>, dim3(grid), dim3(256), 0, s, bt);
            if (kind != 1) {   // the split levels' partials added and applied, one workgroup per tile
              LAUNCH_CHECK();
              SweepBatch bc = bt;
              for (int q2 = 0; q2 <= bt.n; ++q2) bc.first[q2] = bt.first[q2] / cr_split(kind);
              bc.total = bc.first[bt.n];
              if (kind == 0) hipLaunchKernelGGL(k_cr_combine<0>, dim3(bc.total), dim3(256), 0, s, bc);
              else hipLaunchKernelGGL(k_cr_combine<2>, dim3(bc.total), dim3(256), 0, s, bc);
            }
          } else {
            if (kind == 0) hipLaunchKernelGGL((k_cr_solve<R, NSC, 0>), dim3(grid), blkc, smemc, s, bt);
            else if (kind == 1) hipLaunchKernelGGL((k_cr_solve<R, NSC, 1>), dim3(grid), blkc, smemc, s, bt);
            else hipLaunchKernelGGL((k_cr_solve<R, NSC, 2>), dim3(grid), blkc, smemc, s, bt);
            if (cr_split64(kind) > 1) {   // the partials added and applied, one workgroup per tile
              LAUNCH_CHECK();
              SweepBatch bc = bt;
              for (int q2 = 0; q2 <= bt.n; ++q2) bc.first[q2] = bt.first[q2] / cr_split64(kind);
              bc.total = bc.first[bt.n];
              if (kind == 0) hipLaunchKernelGGL((k_cr_combine64<R, NSC, 0>), dim3(bc.total), dim3(256), 0, s, bc);
              else hipLaunchKernelGGL((k_cr_combine64<R, NSC, 2>), dim3(bc.total), dim3(256), 0, s, bc);
            }
          }
          break;
        case 6: hipLaunchKernelGGL(k_cr_stage, dim3(1, tot), dim3(256), 0, s, bt); break;
        default:
          if (fp32) {
            // the separators' scale exponents (item = chunk), then the FP16-split correction
            // (a batch member with one chunk has no separators, no correction and no
            // exponent buffer: it gets no items)
            SweepBatch be = bt;
            int tc = 0, kmax = 1;
            for (int q2 = 0; q2 < bt.n; ++q2) {
              be.first[q2] = tc;
              if (ps[q2]->P > 1) tc += ps[q2]->P;
              kmax = std::max(kmax, ps[q2]->K);
            }
            be.first[bt.n] = be.total = tc;
            hipLaunchKernelGGL(k_corr_exponents, dim3(kmax, tc), dim3(256), 0, s, be);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_correct_h, dim3(grid), dim3(256), 0, s, bt);
          } else {
            hipLaunchKernelGGL(k_correct64_mfma, dim3(grid), dim3(256), 0, s, bt);
          }
      }
      LAUNCH_CHECK();
    }
  }
  return KF_OK;
}

template <typename R, typename IO, bool ADJ>
kf_status solve_copies(const std::vector<kf_problem *> &ps, const IO *const *rhs, IO *const *x, hipStream_t s,
                       int ns, kf_problem *prof) {
  const bool fp32 = sizeof(R) == sizeof(float);
  for (size_t q = 0; q < ps.size(); ++q) {
    kf_problem *p = ps[q];
    const dim3 grid((p->nx + 31) / 32, (p->nz + 31) / 32, p->K);
    hipLaunchKernelGGL((k_to_colmajor<R, IO, ADJ>), grid, dim3(32, 8), 0, s, p->grid(), rhs[q],
                       (cplx<R> *)(fp32 ? (void *)p->sol32 : (void *)p->sol64));
    LAUNCH_CHECK();
  }
  // FP64 sweeps use at most 4 right-hand sides per workgroup (register budget)
  constexpr int NS_MAX = sizeof(R) == 4 ? 8 : 4;
  kf_status st = ns >= 8 ? solve_phases<R, NS_MAX>(ps, s, prof)
               : ns >= 4 ? solve_phases<R, 4>(ps, s, prof)
               : ns >= 2 ? solve_phases<R, 2>(ps, s, prof)
                         : solve_phases<R, 1>(ps, s, prof);
  if (st != KF_OK) return st;
  for (size_t q = 0; q < ps.size(); ++q) {
    kf_problem *p = ps[q];
    const dim3 grid((p->nx + 31) / 32, (p->nz + 31) / 32, p->K);
    hipLaunchKernelGGL((k_from_colmajor<R, IO, ADJ>), grid, dim3(32, 8), 0, s, p->grid(),
                       (const cplx<R> *)(fp32 ? (void *)p->sol32 : (void *)p->sol64), x[q]);
    LAUNCH_CHECK();
  }
  return KF_OK;
}

template <typename R, typename IO>
kf_status solve_dispatch(const std::vector<kf_problem *> &ps, int adjoint, const IO *const *rhs, IO *const *x,
                         hipStream_t s, kf_problem *prof) {
  if ((int)ps.size() > KF_BATCH_MAX) { set_error("batch too large"); return KF_EINVAL; }
  const bool fp32 = sizeof(R) == sizeof(float);
  // sources per workgroup: the choice of the problem with the most work
  int ns = 1;
  double most = -1.0;
  for (kf_problem *p : ps) {
    if (!(fp32 ? p->have_T32 : p->have_T64)) { set_error("block solve before factorisation"); return KF_ESTATE; }
    const double w = (double)p->nx * p->nz * p->nz * p->K;
    if (w > most) { most = w; ns = p->ns; }
  }
  ProfScope sw(prof, PROF_SWEEP);
  return adjoint ? solve_copies<R, IO, true>(ps, rhs, x, s, ns, prof) : solve_copies<R, IO, false>(ps, rhs, x, s, ns, prof);
}
}  // namespace

template <>
kf_status blu_solve<double>(kf_problem *p, int adjoint, const double2 *rhs, double2 *x) {
  kf_status st = blu_factor(p, 1);
  if (st != KF_OK) return st;
  return solve_dispatch<double, double2>({p}, adjoint, &rhs, &x, p->stream, p);
}
template <>
kf_status blu_solve<float>(kf_problem *p, int adjoint, const float2 *rhs, float2 *x) {
  kf_status st = blu_factor(p, 2);
  if (st != KF_OK) return st;
  return solve_dispatch<float, float2>({p}, adjoint, &rhs, &x, p->stream, p);
}
kf_status blu_solve_mixed_io(kf_problem *p, int adjoint, const double2 *rhs, double2 *x) {
  kf_status st = blu_factor(p, 2);
  if (st != KF_OK) return st;
  return solve_dispatch<float, double2>({p}, adjoint, &rhs, &x, p->stream, p);
}

// rhs[q], x[q]: IO-typed fields of problem q; R = double uses the FP64 factors, float
// the complex64 ones.
template <typename R, typename IO>
kf_status blu_solve_batch(const std::vector<kf_problem *> &ps, int adjoint, const IO *const *rhs, IO *const *x,
                          hipStream_t s) {
  return solve_dispatch<R, IO>(ps, adjoint, rhs, x, s, nullptr);
}
template kf_status blu_solve_batch<double, double2>(const std::vector<kf_problem *> &, int, const double2 *const *,
                                                    double2 *const *, hipStream_t);
template kf_status blu_solve_batch<float, double2>(const std::vector<kf_problem *> &, int, const double2 *const *,
                                                   double2 *const *, hipStream_t);
template kf_status blu_solve_batch<float, float2>(const std::vector<kf_problem *> &, int, const float2 *const *,
                                                  float2 *const *, hipStream_t);
