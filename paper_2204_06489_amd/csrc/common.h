// Internal declarations shared by the HIP translation units of libkktfwi.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kktfwi.h"

// ---------------------------------------------------------------------------
// complex arithmetic on interleaved (re, im) pairs
// ---------------------------------------------------------------------------
template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename R> __host__ __device__ inline cplx<R> mk(R re, R im) { cplx<R> c; c.x = re; c.y = im; return c; }
template <typename C> __host__ __device__ inline C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) { C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c; }
// conj(a) * b
template <typename C> __host__ __device__ inline C cmulc(C a, C b) { C c; c.x = a.x * b.x + a.y * b.y; c.y = a.x * b.y - a.y * b.x; return c; }
template <typename C> __host__ __device__ inline C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename R> __host__ __device__ inline C cscale(C a, R s) { a.x *= s; a.y *= s; return a; }
// acc += a * b
template <typename C> __host__ __device__ inline void cfma(C &acc, C a, C b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm keeps the scaling safe for the large PML stretch factors
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
template <typename C> __host__ __device__ inline double cabs2(C a) { return (double)a.x * a.x + (double)a.y * a.y; }

template <typename To, typename From> __device__ inline cplx<To> ccast(From a) { return mk<To>((To)a.x, (To)a.y); }

// ---------------------------------------------------------------------------
// PML and stencil coefficients of one grid (device arrays, c128)
//   xn[i]   = X(x_i)                 i = 0..nx-1
//   ixh[i]  = 1 / X(x_{i-1/2})       i = 0..nx   (faces of node i are ixh[i], ixh[i+1])
//   zn, izh likewise along z
// ---------------------------------------------------------------------------
struct Grid {
  int nx, nz, npml;
  double h, omega;
  const double *gamma;      // [nz][nx]
  const double2 *xn, *ixh, *zn, *izh;
  double beta;              // 0 for A; beta != 0 gives the shifted operator A(gamma (1 + i beta))
};

// The five stencil weights of node (i, j) of A (Section 2, 5-point PML scheme):
//   (A u)_ij = cc u_ij + cxm u_{i-1,j} + cxp u_{i+1,j} + czm u_{i,j-1} + czp u_{i,j+1}
struct Stencil5 { double2 cc, cxm, cxp, czm, czp; };

__device__ inline Stencil5 stencil_at(const Grid &g, int i, int j) {
  const double ih2 = 1.0 / (g.h * g.h);
  const double2 X = g.xn[i], Z = g.zn[j];
  Stencil5 s;
  s.cxm = cscale(cmul(Z, g.ixh[i]), -ih2);
  s.cxp = cscale(cmul(Z, g.ixh[i + 1]), -ih2);
  s.czm = cscale(cmul(X, g.izh[j]), -ih2);
  s.czp = cscale(cmul(X, g.izh[j + 1]), -ih2);
  const double w2g = g.omega * g.omega * g.gamma[(size_t)j * g.nx + i];
  double2 m = cscale(cmul(X, Z), w2g);
  if (g.beta != 0.0) m = cmul(m, make_double2(1.0, g.beta));   // shifted mass term (multigrid levels)
  s.cc = csub(make_double2(0.0, 0.0), cadd(cadd(s.cxm, s.cxp), cadd(s.czm, s.czp)));
  s.cc = csub(s.cc, m);
  return s;
}

// coupling weight between column i-1 and column i at row j (the block-tridiagonal
// off-diagonal C_i of A; A is complex symmetric so it is the same in both directions)
__device__ inline double2 coupling_x(const Grid &g, int i, int j) {
  return cscale(cmul(g.zn[j], g.ixh[i]), -1.0 / (g.h * g.h));
}

// ---------------------------------------------------------------------------
// batch descriptors, passed by value to the persistent work-list kernels
// ---------------------------------------------------------------------------
constexpr int KF_BATCH_MAX = 8;
constexpr int KF_MAX_CHUNKS = 64;   // column chunks of the partitioned factorisation
struct SweepProblem {
  Grid g;
  int K, P, lmax;      // sources, chunks, longest chunk (columns)
  const int *part;     // [P][3]: first, last and meeting column of each chunk (device)
  const void *T, *V, *W;   // factors and spikes (c128 or c64)
  const void *CR;      // separators' reduction blocks ML, MU: [n][levels][2][m][m]
  void *x;             // right-hand sides in, solutions out: column-major [K][nx][nz] (compute type)
  void *gsep;          // the separators' reduced right-hand sides, staged before the
                       // back-substitution: [n][K][m] (complex64 solves)
  const uint16_t *vwh; // the spikes of the interior columns as scaled FP16 pairs (see
  const int *vwe;      //   blocklu.hip, the correction of complex64 solves): values,
  int *corr_e;         //   per-column exponents, per-(chunk, source) exponents
  int k2;              // k range of a row of the FP16 pairs (2 x m rounded up to 32)
  float2 *crp;         // the terms' partials of a split reduction level (complex64 tiles
                       //   [tiles][3][16][64], or FP64 vectors [tiles][3][NS][m])
};
struct SweepBatch {
  int n, total, level;           // level: cyclic-reduction level of the launch
  int first[KF_BATCH_MAX + 1];   // first item of each problem (prefix sums)
  int xs[9];                     // items [xs[x], xs[x+1]) run on XCD x
  SweepProblem p[KF_BATCH_MAX];
};
struct FactorProblem {
  Grid g;
  int P;
  const int *part;
  double2 *T, *V, *W, *work;
  double2 *lu;         // separators' current L, U and staging: [n][4][m][m]
};
struct FactorBatch {
  int n, total;
  int first[KF_BATCH_MAX + 1];
  int xs[9];
  FactorProblem p[KF_BATCH_MAX];
};

// ---------------------------------------------------------------------------
// problem state
// ---------------------------------------------------------------------------
// per kernel family: launches, milliseconds and the algorithmic work of the recorded
// launches (bytes for memory-bound families, flops for the block sweeps; 0 if the
// family does not count it)
struct ProfCounter { int64_t launches = 0; double ms = 0.0, work = 0.0; };

struct kf_problem {
  kf_desc d;                      // copy; its host arrays point into the vectors below
  std::vector<int32_t> src_ix, src_iz, rec_ix, rec_iz;
  std::vector<double> w;          // [K][nrec]
  int nx, nz, npml, K, nrec, nxc, nzc;
  int64_t Nu, Ng, Nxi;
  double h, omega, eps;
  hipStream_t stream = nullptr;

  // device state
  double *gamma = nullptr;                     // [nz][nx]
  double2 *xn = nullptr, *ixh = nullptr, *zn = nullptr, *izh = nullptr;
  int32_t *d_src = nullptr;                    // [K] natural node index of source k
  int32_t *d_rnode = nullptr;                  // [nru] unique receiver nodes
  int nru = 0;
  double *d_wsq = nullptr;                     // [K][nru] sum of w^2 of receivers at a node
  int32_t *d_rec = nullptr;                    // [nrec] natural node of receiver r
  int32_t *d_rptr = nullptr, *d_rlist = nullptr; // receivers of each unique node (CSR)
  double2 *d_r = nullptr, *d_wr = nullptr;     // [K][nrec] data residual and weighted residual
  double *d_w = nullptr;                       // [K][nrec]
  double2 *u_n = nullptr;                      // [K][nz][nx]
  double2 *ys_part = nullptr;                  // [groups][Ng] per-source-group parts of sum_k P_k^* lambda_k
  int kkt_groups_max = 0;
  int kkt_resident = 0;                        // resident k_kkt_apply workgroups on the device
  bool have_un = false;

  // partitioned block factorisation over grid columns
  int P = 0;                                   // chunks
  int ns = 1;                                  // sources per workgroup in the block solves
  int lmax = 1;                                // longest chunk (columns)
  std::vector<int> part;                       // [P][3] first, last, meeting column of each chunk
  int *d_part = nullptr;                       // device copy (KF_MAX_CHUNKS * 3)
  double2 *T64 = nullptr;                      // [nx][nz][nz], T_i stored transposed
  float2 *T32 = nullptr;                       // complex64 copy
  double2 *V64 = nullptr, *W64 = nullptr;      // spikes and separator blocks (P > 1)
  float2 *V32 = nullptr, *W32 = nullptr;
  bool have_T64 = false, have_T32 = false;
  double2 *fac_work = nullptr;                 // factorisation scratch, fac_slots work matrices
  size_t fac_slots = 0;
  double2 *CRL64 = nullptr;                    // separators' L, U during the reduction [n][4][m][m]
  double2 *CR64 = nullptr;                     // separators' ML, MU [n][levels][2][m][m]
  float2 *CR32 = nullptr;
  float2 *sep32 = nullptr;                     // separators' right-hand sides staged by a solve [n][K][m]
  uint16_t *vwh = nullptr;                     // spikes as scaled FP16 (hi, lo) pairs [nx][m][k2 / 8][4][8]
  int *vwe = nullptr;                          // their per-column scale exponents [nx]
  int *corr_e = nullptr;                       // per-(chunk, source) exponents of a solve's separators [P][K]
  float2 *cr_part = nullptr;                   // the terms' partials of a split reduction level
  int vw_k2 = 0;
  void *fac_jobs = nullptr;                    // device job tables of the factorisation
  size_t fac_jobs_cap = 0;                     // bytes
  double2 *sol64 = nullptr;                    // [K][nx][nz] column-major solve copy (c128)
  float2 *sol32 = nullptr;                     // the same for complex64 sweeps

  // scratch
  double2 *vec_a = nullptr, *vec_b = nullptr, *vec_c = nullptr, *vec_d = nullptr;  // [K][nz][nx] each
  double *red = nullptr;                       // reduction partials
  double *red_out = nullptr;                   // small reduction results
  double *host_pinned = nullptr;               // pinned readback buffer

  // Krylov bases (allocated on first use)
  int krylov_m = 0;
  double2 *V = nullptr, *Z = nullptr;          // (m+1) and m packed vectors
  double2 *xi_w = nullptr, *xi_b = nullptr, *xi_x = nullptr;
  double2 *hess = nullptr;                     // (m+1) x m Hessenberg + rotations etc.
  // reduced-space CG (allocated on first use): five control vectors and one field
  double2 *cg_vec = nullptr;                   // [5][Ng]: ds, residual, direction, H direction, g
  double2 *cg_field = nullptr;                 // [K][nz][nx]
  double2 *bicg = nullptr;                     // outer BiCGStab: 8 packed vectors (allocated on first use)
  // H-block of the preconditioner's middle stage: 0 = L = eps I; 1 = L-BFGS from pairs
  // (s_i, H s_i) with L as the initial matrix (a ring of up to hb_max pairs)
  int hblock = 0, hb_max = 0, hb_n = 0, hb_head = 0;
  double2 *hb_s = nullptr, *hb_y = nullptr;    // [hb_max][Ng]
  double2 *hb_q = nullptr;                     // [Ng] work vector of the two-loop recursion
  std::vector<double> hb_rho;                  // 1 / Re(y_i^H s_i)

  double beta = 0.0;                           // mass-term shift (multigrid levels only)
  uint64_t gamma_version = 0;                  // bumped whenever gamma changes
  Grid grid() const { return Grid{nx, nz, npml, h, omega, gamma, xn, ixh, zn, izh, beta}; }

  // shifted-Laplacian multigrid (the third preconditioner variant), built on first use
  struct MgState *mg = nullptr;

  // profiling
  bool prof = false;
  uint32_t prof_mask = ~0u;                    // families recorded (bit = ProfId)
  std::vector<hipEvent_t> ev_free;             // event pool
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[32];   // indexed by ProfId (< 32)
  ProfCounter counters[32];
};

enum ProfId { PROF_KKT = 0, PROF_STENCIL, PROF_FACTOR, PROF_SWEEP, PROF_PRECOND, PROF_ORTH, PROF_REDUCE,
              PROF_FWD64, PROF_FWD32, PROF_BWD64, PROF_BWD32, PROF_MID, PROF_REDRHS, PROF_CHAIN, PROF_CORRECT,
              PROF_GS_DOT, PROF_GS_UPDATE, PROF_MG, PROF_N };
static_assert(PROF_N <= 32, "profiling families are bits of a 32-bit mask");

// error plumbing
void set_error(const std::string &msg);
// hipMalloc of the library's device buffers.  With KF_POISON_ALLOC set in the
// environment every new buffer is filled with 0xFF bytes (NaN in FP32 and FP64), so
// that a read of memory no kernel has written shows up as a NaN instead of depending
// on what the memory held before.
hipError_t kf_malloc(void **ptr, size_t bytes);
#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_));    \
      return KF_EHIP;                                                                    \
    }                                                                                    \
  } while (0)

// profiling helpers (no-ops unless enabled)
struct ProfScope {
  kf_problem *p; int id; hipEvent_t a{}, b{};
  ProfScope(kf_problem *p_, int id_, double work = 0.0);
  ~ProfScope();
};

// ---------------------------------------------------------------------------
// launchers (all enqueue on p->stream)
// ---------------------------------------------------------------------------
kf_status launch_pml(kf_problem *p, const kf_desc &d);
// X (nodes) and 1/X (faces) of one axis of n nodes (the PML stretch of Section 2)
kf_status launch_stretch(hipStream_t s, int n, double h, int npml, double omega, double r0, double cref, double2 *fn,
                         double2 *ifh);
template <typename R> kf_status launch_stencil(kf_problem *p, int adjoint, const cplx<R> *x, cplx<R> *y);
kf_status launch_kkt_apply(kf_problem *p, const double2 *xi, double2 *y);
kf_status launch_kkt_apply_noalloc(kf_problem *p, const double2 *xi, double2 *y);   // scratch array, no allocation
kf_status launch_precond_stage2(kf_problem *p, const double2 *y, double2 *z);
kf_status launch_sources(kf_problem *p, double2 *f);
kf_status launch_residual(kf_problem *p, const double2 *d_obs, const double2 *u, double2 *r, double2 *wr);
kf_status launch_rhs(kf_problem *p, const double2 *r, const int32_t *rptr, const int32_t *rlist, double2 *b,
                     int reg_on_update);
kf_status launch_update_gamma(kf_problem *p, const double2 *ds, double *target);
kf_status launch_grad_gamma(kf_problem *p, const void *u, const void *mu, int c64, double *grad);
kf_status launch_axpy_field(kf_problem *p, int64_t n, double2 a, const double2 *x, double2 *y);
kf_status launch_copy_c128_to_c64(kf_problem *p, int64_t n, const double2 *x, float2 *y);
// y = a x + b y
kf_status launch_axpby_field(kf_problem *p, int64_t n, double2 a, const double2 *x, double2 b, double2 *y);
// reduced Hessian pieces (Section 3): out_k = P_k v; out = Q^T W^2 Q x; out = Q^T W^2 r;
// out = alpha v + P^* lambda + gcoef gamma_core (real part only with real_only)
kf_status launch_scatter_P(kf_problem *p, const double2 *v, double2 *out);
kf_status launch_apply_F(kf_problem *p, const double2 *x, double2 *out);
kf_status launch_rhs_u_field(kf_problem *p, const double2 *r, double2 *out);
kf_status launch_gather_PH(kf_problem *p, double alpha, const double2 *v, double gcoef, const double2 *lam,
                           int real_only, double2 *out);
kf_status launch_copy_c64_to_c128(kf_problem *p, int64_t n, const float2 *x, double2 *y);

// shifted-Laplacian multigrid (multigrid.hip)
kf_status mg_configure(kf_problem *p, int prec, double beta, double rtol, int maxit, int n_min);
// BiCGStab with one V-cycle per preconditioning step; b and x (c128) may alias; rtol / maxit
// <= 0 take the configured values
kf_status mg_solve(kf_problem *p, int adjoint, const double2 *b, double2 *x, double rtol, int maxit, kf_mg_stats *st);
kf_status mg_vcycle_apply(kf_problem *p, const double2 *b, double2 *x);
int mg_levels(kf_problem *p, int *dims);
void mg_destroy(kf_problem *p);

// block factorisation and sweeps
int blu_auto_chunks(int nx, int nz, int K);
kf_status blu_set_shape(kf_problem *p, int chunks, int ns);   // chunks 0 = automatic, ns 0 = 1
kf_status blu_factor(kf_problem *p, int which);
template <typename R> kf_status blu_solve(kf_problem *p, int adjoint, const cplx<R> *rhs, cplx<R> *x);
kf_status blu_solve_mixed_io(kf_problem *p, int adjoint, const double2 *rhs, double2 *x);  // c64 factors, c128 I/O

// batches: persistent work-list kernels over several problems (one launch per phase)
kf_status blu_factor_batch(const std::vector<kf_problem *> &ps, int which, hipStream_t s);
template <typename R, typename IO>
kf_status blu_solve_batch(const std::vector<kf_problem *> &ps, int adjoint, const IO *const *rhs, IO *const *x,
                          hipStream_t s);

// reductions (deterministic, fixed order)
kf_status per_source_norms(kf_problem *p, const double2 *x, int64_t n_per, int K, double *out_host);
// number of NaN / inf entries of a real device array (synchronises the stream)
kf_status count_nonfinite(kf_problem *p, const double *a, int64_t n, int64_t *count_host);
kf_status dot_c128(kf_problem *p, const double2 *a, const double2 *b, int64_t n, double2 *out_dev);
// `active` (device int, may be NULL): the launch does nothing when *active == 0
kf_status norm_c128(kf_problem *p, const double2 *a, int64_t n, double *out_dev, const int *active = nullptr);
// h_dev = V^H w (nv vectors); with nrm2_out also |w|^2 from the same sweep
kf_status multidot_c128(kf_problem *p, const double2 *V, int nv, const double2 *w, int64_t n, double2 *h_dev,
                        const int *active = nullptr, double *nrm2_out = nullptr);
kf_status multiaxpy_c128(kf_problem *p, const double2 *V, int nv, const double2 *h_dev, double sign, double2 *w,
                         int64_t n, const int *active = nullptr);
// w <- (w - V h) * scale[0] (scale NULL: 1), then nrm_out = |w| and the first
// min(nv, 8) entries of h_out = V^H w (h_out may be NULL), in one sweep over V;
// multidot_rest_c128 gives the other entries.  With scale the update itself always
// runs and `active` gates only the norm; `active_dots` (if given) gates the dots.
kf_status axpy_dot_c128(kf_problem *p, const double2 *V, int nv, const double2 *h, double2 *w, int64_t n,
                        double2 *h_out, double *nrm_out, const int *active = nullptr,
                        const double *scale = nullptr, const int *active_dots = nullptr);
// Gram-Schmidt decision from |w|^2 and h1 = V^H w before the first update (see krylov.hip)
kf_status gs_decide(kf_problem *p, int nv, const double2 *h1, const double *wn2, double eta, double2 *h2, int *flags,
                    double *nrm, double *scale);
kf_status multidot_rest_c128(kf_problem *p, const double2 *V, int nv, const double2 *w, int64_t n, double2 *h_out,
                             const int *active = nullptr);
// FGMRES small dense algebra on the device (single-thread kernels)
kf_status arnoldi_finish(kf_problem *p, int j, int m, const double2 *h1, const double2 *h2, const double *nrm,
                         double2 *H, double2 *cs, double2 *sn, double2 *g, double *resid);
kf_status scale_inv(kf_problem *p, int64_t n, const double *nrm, const double2 *x, double2 *y,
                    const int *active = nullptr);
kf_status hess_backsolve(kf_problem *p, int nj, int m, const double2 *H, const double2 *g, double2 *y);
kf_status set_g0(kf_problem *p, int m, const double *beta, double2 *g);
kf_status imag_part(kf_problem *p, int64_t n, const double2 *x, double2 *y);
