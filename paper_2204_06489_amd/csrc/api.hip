// C ABI of libkktfwi: validation, device state, Helmholtz block solves, the KKT
// operator and preconditioner, flexible GMRES and the Gauss-Newton step.
#include "common.h"

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <tuple>

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

hipError_t kf_malloc(void **ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e == hipSuccess && std::getenv("KF_POISON_ALLOC")) {
    e = hipMemset(*ptr, 0xFF, bytes);
    if (e != hipSuccess) {
      (void)hipFree(*ptr);
      *ptr = nullptr;
    }
  }
  return e;
}
static kf_status fail(kf_status st, const std::string &msg) {
  set_error(msg);
  return st;
}
#define CHECK_ST(expr)                  \
  do {                                  \
    kf_status s_ = (expr);              \
    if (s_ != KF_OK) return s_;         \
  } while (0)

extern "C" const char *kf_version(void) { return "kktfwi 0.1 (gfx950)"; }
extern "C" const char *kf_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// profiling: HIP events around launches of a kernel family, from a pool
// ---------------------------------------------------------------------------
static hipEvent_t take_event(kf_problem *p) {
  if (p->ev_free.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = p->ev_free.back();
  p->ev_free.pop_back();
  return e;
}
ProfScope::ProfScope(kf_problem *p_, int id_, double work) : p(p_), id(id_) {
  if (!p || id < 0 || !p->prof || !((p->prof_mask >> id) & 1u)) return;
  p->counters[id].work += work;
  a = take_event(p);
  b = take_event(p);
  if (a) hipEventRecord(a, p->stream);
}
ProfScope::~ProfScope() {
  if (!p || id < 0 || !p->prof || !a || !b) return;
  hipEventRecord(b, p->stream);
  p->pending[id].push_back({a, b});
}
static void prof_collect(kf_problem *p) {
  bool any = false;
  for (int i = 0; i < PROF_N; ++i) any |= !p->pending[i].empty();
  if (!any) return;
  hipStreamSynchronize(p->stream);
  for (int i = 0; i < PROF_N; ++i) {
    for (auto &pr : p->pending[i]) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, pr.first, pr.second);
      p->counters[i].launches += 1;
      p->counters[i].ms += ms;
      p->ev_free.push_back(pr.first);
      p->ev_free.push_back(pr.second);
    }
    p->pending[i].clear();
  }
}

// phase timer for the Newton-step breakdown (events, summed at the end)
struct PhaseTimer {
  kf_problem *p;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> recs;
  int cur = -1;
  hipEvent_t cur_a = nullptr;
  explicit PhaseTimer(kf_problem *p_) : p(p_) {}
  void start(int phase) {
    cur = phase;
    cur_a = take_event(p);
    if (cur_a) hipEventRecord(cur_a, p->stream);
  }
  void stop() {
    hipEvent_t b = take_event(p);
    if (b && cur_a) {
      hipEventRecord(b, p->stream);
      recs.push_back({cur, {cur_a, b}});
    }
    cur_a = nullptr;
  }
  void sum(double *out, int n) {
    hipStreamSynchronize(p->stream);
    for (auto &r : recs) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, r.second.first, r.second.second);
      if (r.first < n) out[r.first] += ms;
      p->ev_free.push_back(r.second.first);
      p->ev_free.push_back(r.second.second);
    }
    recs.clear();
  }
};
enum { PH_PRECOND = 0, PH_MATVEC, PH_ORTH, PH_N };

// ---------------------------------------------------------------------------
// allocation helpers
// ---------------------------------------------------------------------------
template <typename T> static kf_status dalloc(T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = kf_malloc((void **)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(KF_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes failed: " +
                               hipGetErrorString(e));
  }
  return KF_OK;
}
template <typename T> static void dfree(T *&ptr) {
  if (ptr) hipFree((void *)ptr);
  ptr = nullptr;
}

static void free_all(kf_problem *p) {
  dfree(p->gamma); dfree(p->xn); dfree(p->ixh); dfree(p->zn); dfree(p->izh);
  dfree(p->d_src); dfree(p->d_rnode); dfree(p->d_wsq); dfree(p->d_rec); dfree(p->d_w);
  dfree(p->d_rptr); dfree(p->d_rlist); dfree(p->d_r); dfree(p->d_wr);
  dfree(p->u_n); dfree(p->ys_part); dfree(p->T64); dfree(p->T32); dfree(p->fac_work); dfree(p->d_part); dfree(p->sol64); dfree(p->sol32);
  dfree(p->CRL64); dfree(p->CR64); dfree(p->CR32); dfree(p->sep32); dfree(p->vwh); dfree(p->vwe);
  dfree(p->corr_e); dfree(p->cr_part);
  if (p->fac_jobs) hipFree(p->fac_jobs);
  dfree(p->V64); dfree(p->W64); dfree(p->V32); dfree(p->W32);
  dfree(p->vec_a); dfree(p->vec_b); dfree(p->vec_c); dfree(p->vec_d); dfree(p->red); dfree(p->red_out);
  dfree(p->V); dfree(p->Z); dfree(p->xi_w); dfree(p->xi_b); dfree(p->xi_x); dfree(p->hess);
  dfree(p->cg_vec); dfree(p->cg_field); dfree(p->bicg);
  dfree(p->hb_s); dfree(p->hb_y); dfree(p->hb_q);
  mg_destroy(p);
  if (p->host_pinned) hipHostFree(p->host_pinned);
  p->host_pinned = nullptr;
  for (int i = 0; i < PROF_N; ++i) {
    for (auto &pr : p->pending[i]) { hipEventDestroy(pr.first); hipEventDestroy(pr.second); }
    p->pending[i].clear();
  }
  for (auto e : p->ev_free) hipEventDestroy(e);
  p->ev_free.clear();
}

// ---------------------------------------------------------------------------
// validation (no HIP calls)
// ---------------------------------------------------------------------------
static const int MAX_NZ = 512;   // column block size held by the factorisation kernels

static kf_status validate_desc(const kf_desc *d) {
  if (!d) return fail(KF_EINVAL, "desc is NULL");
  if (d->nx < 3 || d->nz < 3) return fail(KF_ESHAPE, "nx and nz must be >= 3");
  if (d->nz > MAX_NZ) return fail(KF_ESHAPE, "nz must be <= 512 (column block of the factorisation)");
  if ((int64_t)d->nx * d->nz > (int64_t)1 << 31) return fail(KF_ESHAPE, "grid too large");
  if (!(d->h > 0.0) || !std::isfinite(d->h)) return fail(KF_EINVAL, "h must be > 0");
  if (d->npml < 0 || 2 * d->npml >= d->nx || 2 * d->npml >= d->nz)
    return fail(KF_EINVAL, "npml must satisfy 0 <= 2*npml < min(nx, nz)");
  if (d->npml > 0 && !(d->pml_r0 > 0.0 && d->pml_r0 < 1.0)) return fail(KF_EINVAL, "pml_r0 must be in (0, 1)");
  if (d->npml > 0 && !(d->pml_cref > 0.0 && std::isfinite(d->pml_cref))) return fail(KF_EINVAL, "pml_cref must be > 0");
  if (!(d->omega > 0.0) || !std::isfinite(d->omega)) return fail(KF_EINVAL, "omega must be > 0");
  if (d->K < 1) return fail(KF_EINVAL, "K must be >= 1");
  if (!d->src_ix || !d->src_iz) return fail(KF_EINVAL, "source index arrays are NULL");
  if (d->nrec < 1) return fail(KF_EINVAL, "nrec must be >= 1");
  if (!d->rec_ix || !d->rec_iz) return fail(KF_EINVAL, "receiver index arrays are NULL");
  if (!(d->eps > 0.0) || !std::isfinite(d->eps))
    return fail(KF_EINVAL, "eps must be > 0 (the preconditioner applies L^-1 = I/eps)");
  for (int k = 0; k < d->K; ++k)
    if (d->src_ix[k] < 0 || d->src_ix[k] >= d->nx || d->src_iz[k] < 0 || d->src_iz[k] >= d->nz)
      return fail(KF_EINVAL, "source " + std::to_string(k) + " is off the grid");
  for (int r = 0; r < d->nrec; ++r)
    if (d->rec_ix[r] < 0 || d->rec_ix[r] >= d->nx || d->rec_iz[r] < 0 || d->rec_iz[r] >= d->nz)
      return fail(KF_EINVAL, "receiver " + std::to_string(r) + " is off the grid");
  if (d->w)
    for (int64_t q = 0; q < (int64_t)d->K * d->nrec; ++q)
      if (!std::isfinite(d->w[q])) return fail(KF_EINVAL, "weights must be finite");
  return KF_OK;
}

static kf_status check_p(kf_problem *p) {
  if (!p) return fail(KF_EINVAL, "problem is NULL");
  return KF_OK;
}

// ---------------------------------------------------------------------------
// create / destroy / state
// ---------------------------------------------------------------------------
kf_status tuned_shape(const kf_problem *p, int prec, int *chunks, int *ns);

extern "C" kf_status kf_create(const kf_desc *desc, const double *gamma, int32_t gamma_on_device, void *hip_stream,
                               kf_problem **out) {
  if (!out) return fail(KF_EINVAL, "out is NULL");
  *out = nullptr;
  CHECK_ST(validate_desc(desc));
  if (!gamma) return fail(KF_EINVAL, "gamma is NULL");
  if (!gamma_on_device) {
    for (int64_t q = 0; q < (int64_t)desc->nx * desc->nz; ++q)
      if (!std::isfinite(gamma[q])) return fail(KF_EINVAL, "gamma must be finite");
  }
  kf_problem *p = new kf_problem();
  p->d = *desc;
  p->nx = desc->nx; p->nz = desc->nz; p->npml = desc->npml; p->K = desc->K; p->nrec = desc->nrec;
  p->nxc = p->nx - 2 * p->npml; p->nzc = p->nz - 2 * p->npml;
  p->Nu = (int64_t)p->nx * p->nz; p->Ng = (int64_t)p->nxc * p->nzc; p->Nxi = 2 * p->K * p->Nu + p->Ng;
  p->h = desc->h; p->omega = desc->omega; p->eps = desc->eps;
  p->stream = (hipStream_t)hip_stream;
  p->src_ix.assign(desc->src_ix, desc->src_ix + p->K);
  p->src_iz.assign(desc->src_iz, desc->src_iz + p->K);
  p->rec_ix.assign(desc->rec_ix, desc->rec_ix + p->nrec);
  p->rec_iz.assign(desc->rec_iz, desc->rec_iz + p->nrec);
  p->w.assign((size_t)p->K * p->nrec, 1.0);
  if (desc->w) std::copy(desc->w, desc->w + (size_t)p->K * p->nrec, p->w.begin());
  p->d.src_ix = p->src_ix.data(); p->d.src_iz = p->src_iz.data();
  p->d.rec_ix = p->rec_ix.data(); p->d.rec_iz = p->rec_iz.data(); p->d.w = p->w.data();

  // receivers: natural node of each, unique nodes, CSR lists and summed W^2 per node
  std::vector<int32_t> rec(p->nrec), src(p->K);
  for (int r = 0; r < p->nrec; ++r) rec[r] = p->rec_iz[r] * p->nx + p->rec_ix[r];
  for (int k = 0; k < p->K; ++k) src[k] = p->src_iz[k] * p->nx + p->src_ix[k];
  std::map<int32_t, std::vector<int32_t>> bynode;
  for (int r = 0; r < p->nrec; ++r) bynode[rec[r]].push_back(r);
  std::vector<int32_t> rnode, rptr(1, 0), rlist;
  for (auto &kv : bynode) {
    rnode.push_back(kv.first);
    for (int r : kv.second) rlist.push_back(r);
    rptr.push_back((int32_t)rlist.size());
  }
  p->nru = (int)rnode.size();
  std::vector<double> wsq((size_t)p->K * p->nru, 0.0);
  for (int k = 0; k < p->K; ++k)
    for (int u = 0; u < p->nru; ++u)
      for (int e = rptr[u]; e < rptr[u + 1]; ++e) {
        double ww = p->w[(size_t)k * p->nrec + rlist[e]];
        wsq[(size_t)k * p->nru + u] += ww * ww;
      }

  const size_t Nu = p->Nu, K = p->K, m = p->nz;
  kf_status st = KF_OK;
#define ALLOC(ptr, n) if (st == KF_OK) st = dalloc(&(ptr), (n))
  ALLOC(p->gamma, Nu);
  ALLOC(p->xn, (size_t)p->nx); ALLOC(p->ixh, (size_t)p->nx + 1);
  ALLOC(p->zn, (size_t)p->nz); ALLOC(p->izh, (size_t)p->nz + 1);
  ALLOC(p->d_src, K); ALLOC(p->d_rnode, (size_t)p->nru); ALLOC(p->d_wsq, K * p->nru);
  ALLOC(p->d_rec, (size_t)p->nrec); ALLOC(p->d_w, K * p->nrec);
  ALLOC(p->d_rptr, (size_t)p->nru + 1); ALLOC(p->d_rlist, (size_t)p->nrec);
  ALLOC(p->d_r, K * p->nrec); ALLOC(p->d_wr, K * p->nrec);
  ALLOC(p->u_n, K * Nu);
  p->kkt_groups_max = (int)std::min<size_t>(K, 64);
  ALLOC(p->ys_part, (size_t)p->kkt_groups_max * p->Ng);
  // complex64 factors padded by four zero columns: the matrix-core sweeps read whole
  // k-steps of four columns past a block's end
  ALLOC(p->T64, (size_t)p->nx * m * m); ALLOC(p->T32, (size_t)p->nx * m * m + 4 * m);
  if (st == KF_OK && hipMemset(p->T32 + (size_t)p->nx * m * m, 0, sizeof(float2) * 4 * m) != hipSuccess)
    st = fail(KF_EHIP, "hipMemset failed");
  ALLOC(p->d_part, 3 * KF_MAX_CHUNKS);
  ALLOC(p->sol64, K * Nu); ALLOC(p->sol32, K * Nu);
  ALLOC(p->vec_a, K * Nu); ALLOC(p->vec_b, K * Nu); ALLOC(p->vec_c, K * Nu); ALLOC(p->vec_d, K * Nu);
  ALLOC(p->red, (size_t)1024 * 2 * 256 + K * 64);
  ALLOC(p->red_out, std::max<size_t>(K, 1024));
#undef ALLOC
  if (st == KF_OK && hipHostMalloc((void **)&p->host_pinned, sizeof(double) * std::max<size_t>(K, 1024)) != hipSuccess) {
    p->host_pinned = nullptr;
    st = fail(KF_ENOMEM, "hipHostMalloc failed");
  }
  if (st != KF_OK) { free_all(p); delete p; return st; }

  auto h2d = [&](void *dst, const void *srcp, size_t bytes) -> kf_status {
    HIP_TRY(hipMemcpyAsync(dst, srcp, bytes, hipMemcpyHostToDevice, p->stream));
    return KF_OK;
  };
  st = h2d(p->d_src, src.data(), sizeof(int32_t) * K);
  if (st == KF_OK) st = h2d(p->d_rec, rec.data(), sizeof(int32_t) * p->nrec);
  if (st == KF_OK) st = h2d(p->d_rnode, rnode.data(), sizeof(int32_t) * p->nru);
  if (st == KF_OK) st = h2d(p->d_rptr, rptr.data(), sizeof(int32_t) * (p->nru + 1));
  if (st == KF_OK) st = h2d(p->d_rlist, rlist.data(), sizeof(int32_t) * p->nrec);
  if (st == KF_OK) st = h2d(p->d_wsq, wsq.data(), sizeof(double) * K * p->nru);
  if (st == KF_OK) st = h2d(p->d_w, p->w.data(), sizeof(double) * K * p->nrec);
  if (st == KF_OK && gamma_on_device) {   // a device gamma is checked on the device before it is copied
    int64_t bad = 0;
    st = count_nonfinite(p, gamma, (int64_t)Nu, &bad);
    if (st == KF_OK && bad) st = fail(KF_EINVAL, "gamma must be finite (" + std::to_string(bad) + " NaN/inf entries)");
  }
  if (st == KF_OK) {
    hipError_t e = hipMemcpyAsync(p->gamma, gamma, sizeof(double) * Nu,
                                  gamma_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) st = fail(KF_EHIP, std::string("copy of gamma failed: ") + hipGetErrorString(e));
  }
  if (st == KF_OK) st = launch_pml(p, p->d);
  if (st == KF_OK && hipStreamSynchronize(p->stream) != hipSuccess) st = fail(KF_EHIP, "stream synchronize failed");
  if (st == KF_OK) {   // the shape the autotuner found for this size, if any
    int c = 0, ns = 0;
    if (tuned_shape(p, KF_C64, &c, &ns) != KF_OK) tuned_shape(p, KF_C128, &c, &ns);
    st = blu_set_shape(p, c, ns);
  }
  if (st != KF_OK) { free_all(p); delete p; return st; }
  *out = p;
  return KF_OK;
}

extern "C" kf_status kf_destroy(kf_problem *p) {
  if (!p) return KF_OK;
  hipStreamSynchronize(p->stream);
  free_all(p);
  delete p;
  return KF_OK;
}

extern "C" kf_status kf_set_stream(kf_problem *p, void *s) {
  CHECK_ST(check_p(p));
  p->stream = (hipStream_t)s;
  return KF_OK;
}

extern "C" kf_status kf_set_solver_shape(kf_problem *p, int32_t chunks, int32_t sources_per_group) {
  CHECK_ST(check_p(p));
  return blu_set_shape(p, chunks, sources_per_group);
}

extern "C" kf_status kf_get_solver_shape(kf_problem *p, int32_t *chunks, int32_t *sources_per_group) {
  CHECK_ST(check_p(p));
  if (chunks) *chunks = p->P;
  if (sources_per_group) *sources_per_group = p->ns;
  return KF_OK;
}

extern "C" kf_status kf_set_gamma(kf_problem *p, const double *gamma) {
  CHECK_ST(check_p(p));
  if (!gamma) return fail(KF_EINVAL, "gamma is NULL");
  // checked before it replaces the problem's gamma: a NaN or inf must never reach the
  // factorisation (the problem keeps its previous gamma and factors on failure)
  int64_t bad = 0;
  CHECK_ST(count_nonfinite(p, gamma, p->Nu, &bad));
  if (bad) return fail(KF_EINVAL, "gamma must be finite (" + std::to_string(bad) + " NaN/inf entries)");
  HIP_TRY(hipMemcpyAsync(p->gamma, gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
  p->have_T64 = p->have_T32 = false;
  ++p->gamma_version;
  p->have_un = false;
  return KF_OK;
}

extern "C" kf_status kf_get_gamma(kf_problem *p, double *out) {
  CHECK_ST(check_p(p));
  if (!out) return fail(KF_EINVAL, "output is NULL");
  HIP_TRY(hipMemcpyAsync(out, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
  return KF_OK;
}

extern "C" kf_status kf_set_background(kf_problem *p, const void *u) {
  CHECK_ST(check_p(p));
  if (!u) return fail(KF_EINVAL, "u_n is NULL");
  HIP_TRY(hipMemcpyAsync(p->u_n, u, sizeof(double2) * p->K * p->Nu, hipMemcpyDeviceToDevice, p->stream));
  p->have_un = true;
  return KF_OK;
}

extern "C" kf_status kf_get_background(kf_problem *p, void *out) {
  CHECK_ST(check_p(p));
  if (!out) return fail(KF_EINVAL, "output is NULL");
  if (!p->have_un) return fail(KF_ESTATE, "no background field");
  HIP_TRY(hipMemcpyAsync(out, p->u_n, sizeof(double2) * p->K * p->Nu, hipMemcpyDeviceToDevice, p->stream));
  return KF_OK;
}

extern "C" kf_status kf_factor(kf_problem *p, int32_t which, double *t_ms) {
  CHECK_ST(check_p(p));
  if (which < 1 || which > 3) return fail(KF_EINVAL, "which must be 1, 2 or 3");
  HIP_TRY(hipStreamSynchronize(p->stream));
  auto t0 = std::chrono::steady_clock::now();
  CHECK_ST(blu_factor(p, which));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (t_ms) *t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return KF_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the block solver's shape (chunks x sources per workgroup)
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int nx, nz, K, prec;
  bool operator<(const TuneKey &o) const {
    return std::tie(nx, nz, K, prec) < std::tie(o.nx, o.nz, o.K, o.prec);
  }
};
std::map<TuneKey, std::pair<int, int>> &tune_cache() {
  static std::map<TuneKey, std::pair<int, int>> c;
  return c;
}

// ms between two events recorded on p->stream around fn()
template <typename F> kf_status timed(kf_problem *p, F fn, double *ms) {
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return fail(KF_EHIP, "hipEventCreate failed"); }
  kf_status st = KF_OK;
  if (hipEventRecord(a, p->stream) != hipSuccess) st = fail(KF_EHIP, "hipEventRecord failed");
  if (st == KF_OK) st = fn();
  if (st == KF_OK && hipEventRecord(b, p->stream) != hipSuccess) st = fail(KF_EHIP, "hipEventRecord failed");
  if (st == KF_OK && hipEventSynchronize(b) != hipSuccess) st = fail(KF_EHIP, "hipEventSynchronize failed");
  float f = 0.f;
  if (st == KF_OK && hipEventElapsedTime(&f, a, b) != hipSuccess) st = fail(KF_EHIP, "hipEventElapsedTime failed");
  hipEventDestroy(a);
  hipEventDestroy(b);
  *ms = f;
  return st;
}
}  // namespace

kf_status tuned_shape(const kf_problem *p, int prec, int *chunks, int *ns) {
  auto it = tune_cache().find(TuneKey{p->nx, p->nz, p->K, prec});
  if (it == tune_cache().end()) return KF_EINVAL;
  *chunks = it->second.first;
  *ns = it->second.second;
  return KF_OK;
}

extern "C" kf_status kf_autotune(kf_problem *p, int32_t prec, double solves_per_factor, kf_tune_entry *table,
                                 int32_t table_len, int32_t *n_table) {
  CHECK_ST(check_p(p));
  if (prec != KF_C128 && prec != KF_C64) return fail(KF_EINVAL, "prec must be KF_C128 or KF_C64");
  if (!(solves_per_factor >= 0.0) || !std::isfinite(solves_per_factor))
    return fail(KF_EINVAL, "solves_per_factor must be >= 0");
  if (table_len < 0 || (table_len > 0 && !table)) return fail(KF_EINVAL, "table is NULL");
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int pmax = std::min(KF_MAX_CHUNKS, (p->nx + 1) / 2);
  const int a = std::max(1, (int)std::lround(1.6 * std::sqrt((double)p->nx)));
  std::vector<int> cand;
  for (double f : {0.0, 0.35, 0.5, 0.7, 1.0, 1.4, 2.0}) {
    int c = f == 0.0 ? 1 : std::max(1, std::min(pmax, (int)std::lround(f * a)));
    if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
  }
  const int64_t n = (int64_t)p->K * p->Nu;
  HIP_TRY(hipMemsetAsync(p->vec_a, 0, sizeof(double2) * n, p->stream));
  const int which = prec == KF_C64 ? 3 : 1;
  auto solve = [&](int adj) -> kf_status {
    return prec == KF_C64 ? blu_solve_mixed_io(p, adj, p->vec_a, p->vec_b) : blu_solve<double>(p, adj, p->vec_a, p->vec_b);
  };
  int count = 0, best_c = 1, best_ns = 1;
  double best = INFINITY;
  auto eval = [&](int c) -> kf_status {
    CHECK_ST(blu_set_shape(p, c, 1));
    double tf = 0.0;
    CHECK_ST(timed(p, [&]() { return blu_factor(p, which); }, &tf));
    for (int ns : {1, 2, 4, 8}) {
      if (ns > 1 && (ns + 1) / 2 >= p->K) break;   // no group would be filled
      CHECK_ST(blu_set_shape(p, c, ns));
      CHECK_ST(solve(0));   // warm-up (first launch of this kernel shape)
      double ts = 0.0;
      CHECK_ST(timed(p, [&]() {
        for (int r = 0; r < 2; ++r) {
          kf_status st = solve(0);
          if (st == KF_OK) st = solve(1);
          if (st != KF_OK) return st;
        }
        return KF_OK;
      }, &ts));
      ts /= 4.0;
      const double score = tf + solves_per_factor * ts;
      if (count < table_len) table[count] = kf_tune_entry{c, ns, tf, ts, score};
      ++count;
      if (score < best) { best = score; best_c = c; best_ns = ns; }
    }
    return KF_OK;
  };
  for (int c : cand) CHECK_ST(eval(c));
  // a finer look around the best chunk count of the grid above (whose steps are ~1.4x):
  // the solve's phases change in steps of their own (e.g. where the sweeps' items pass
  // the number of compute units).  A count found there replaces the grid's best only
  // if it scores more than 2% better: below that, isolated solves do not tell which
  // shape is faster inside a Newton step (at 401x141x40, 34 chunks scored up to 1.7%
  // better than 32 and made the step 7% slower)
  const int c0 = best_c, ns0 = best_ns;
  const double s0 = best;
  for (int c : {c0 - 2, c0 - 1, c0 + 1, c0 + 2})
    if (c > 1 && c <= pmax && 2 * c - 1 <= p->nx && std::find(cand.begin(), cand.end(), c) == cand.end()) {
      cand.push_back(c);
      CHECK_ST(eval(c));
    }
  if (!(best < 0.98 * s0)) {
    best_c = c0;
    best_ns = ns0;
  }
  CHECK_ST(blu_set_shape(p, best_c, best_ns));
  tune_cache()[TuneKey{p->nx, p->nz, p->K, prec}] = {best_c, best_ns};
  if (n_table) *n_table = count;
  return KF_OK;
}

extern "C" kf_status kf_sizes(kf_problem *p, int64_t *out) {
  CHECK_ST(check_p(p));
  if (!out) return fail(KF_EINVAL, "output is NULL");
  out[0] = p->nx; out[1] = p->nz; out[2] = p->K; out[3] = p->nrec; out[4] = p->Ng; out[5] = p->Nxi;
  return KF_OK;
}

extern "C" kf_status kf_sources(kf_problem *p, void *f) {
  CHECK_ST(check_p(p));
  if (!f) return fail(KF_EINVAL, "f is NULL");
  return launch_sources(p, (double2 *)f);
}

extern "C" kf_status kf_stencil_apply(kf_problem *p, int32_t adjoint, int32_t prec, const void *x, void *y) {
  CHECK_ST(check_p(p));
  if (!x || !y) return fail(KF_EINVAL, "x or y is NULL");
  if (x == y) return fail(KF_EINVAL, "x and y must not alias");
  if (prec == KF_C128) return launch_stencil<double>(p, adjoint, (const double2 *)x, (double2 *)y);
  if (prec == KF_C64) return launch_stencil<float>(p, adjoint, (const float2 *)x, (float2 *)y);
  return fail(KF_EINVAL, "prec must be KF_C128 or KF_C64");
}

// ---------------------------------------------------------------------------
// Helmholtz block solves
// ---------------------------------------------------------------------------
// max_k ||rhs_k - op(A) x_k|| / ||rhs_k|| in FP64 (x, rhs c128); uses vec_a, vec_b
static kf_status residual_max(kf_problem *p, int adjoint, const double2 *rhs, const double2 *x, double *relmax,
                              std::vector<double> *rn_cache) {
  const int64_t n = (int64_t)p->K * p->Nu;
  std::vector<double> rn(p->K), bn(p->K);
  if (rn_cache && !rn_cache->empty()) bn = *rn_cache;
  else {
    CHECK_ST(per_source_norms(p, rhs, p->Nu, p->K, bn.data()));
    if (rn_cache) *rn_cache = bn;
  }
  CHECK_ST(launch_stencil<double>(p, adjoint, x, p->vec_a));
  HIP_TRY(hipMemcpyAsync(p->vec_b, rhs, sizeof(double2) * n, hipMemcpyDeviceToDevice, p->stream));
  CHECK_ST(launch_axpy_field(p, n, make_double2(-1.0, 0.0), p->vec_a, p->vec_b));
  CHECK_ST(per_source_norms(p, p->vec_b, p->Nu, p->K, rn.data()));
  double mx = 0.0;
  for (int k = 0; k < p->K; ++k) {
    double r = bn[k] > 0.0 ? rn[k] / bn[k] : rn[k];
    if (!std::isfinite(r)) return fail(KF_ENAN, "non-finite residual in block solve");
    mx = std::max(mx, r);
  }
  *relmax = mx;
  return KF_OK;
}

// complex64 sweeps inside FP64 iterative refinement (x, rhs c128; rhs may alias x)
static kf_status solve_mixed(kf_problem *p, int adjoint, const double2 *rhs, double2 *x, double rtol, int maxit,
                             int *iters, double *relmax) {
  const int64_t n = (int64_t)p->K * p->Nu;
  if (rhs == x) {
    HIP_TRY(hipMemcpyAsync(p->vec_c, rhs, sizeof(double2) * n, hipMemcpyDeviceToDevice, p->stream));
    rhs = p->vec_c;
  }
  CHECK_ST(blu_solve_mixed_io(p, adjoint, rhs, x));
  int it = 1;
  std::vector<double> bn;
  double rm = 0.0;
  for (;;) {
    CHECK_ST(residual_max(p, adjoint, rhs, x, &rm, &bn));   // residual left in vec_b
    if (rm <= rtol || it >= maxit) break;
    CHECK_ST(blu_solve_mixed_io(p, adjoint, p->vec_b, p->vec_a));
    CHECK_ST(launch_axpy_field(p, n, make_double2(1.0, 0.0), p->vec_a, x));
    ++it;
  }
  *iters = it;
  *relmax = rm;
  if (rm > rtol) return fail(KF_ENOCONV, "mixed-precision refinement did not reach rtol");
  return KF_OK;
}

extern "C" kf_status helmholtz_solve(kf_problem *p, int32_t adjoint, int32_t prec, const void *rhs, void *x,
                                     double rtol, int32_t maxit, kf_solve_stats *st) {
  CHECK_ST(check_p(p));
  if (!rhs || !x) return fail(KF_EINVAL, "rhs or x is NULL");
  if (prec != KF_C128 && prec != KF_C64 && prec != KF_MIXED) return fail(KF_EINVAL, "invalid precision");
  if (prec == KF_MIXED && !(rtol > 0.0)) return fail(KF_EINVAL, "KF_MIXED needs rtol > 0");
  if (maxit < 1) maxit = 1;
  const int64_t n = (int64_t)p->K * p->Nu;
  int iters = 1;
  double rm = -1.0;
  kf_status res = KF_OK;
  if (prec == KF_C128) {
    CHECK_ST(blu_solve<double>(p, adjoint, (const double2 *)rhs, (double2 *)x));
    if (rtol > 0.0) {
      if (rhs == x) return fail(KF_EINVAL, "residual report needs rhs and x distinct");
      CHECK_ST(residual_max(p, adjoint, (const double2 *)rhs, (const double2 *)x, &rm, nullptr));
    }
  } else if (prec == KF_C64) {
    CHECK_ST(blu_solve<float>(p, adjoint, (const float2 *)rhs, (float2 *)x));
    if (rtol > 0.0) {
      if (rhs == x) return fail(KF_EINVAL, "residual report needs rhs and x distinct");
      CHECK_ST(launch_copy_c64_to_c128(p, n, (const float2 *)rhs, p->vec_c));
      CHECK_ST(launch_copy_c64_to_c128(p, n, (const float2 *)x, p->vec_d));
      CHECK_ST(residual_max(p, adjoint, p->vec_c, p->vec_d, &rm, nullptr));
    }
  } else {
    res = solve_mixed(p, adjoint, (const double2 *)rhs, (double2 *)x, rtol, maxit, &iters, &rm);
    if (res != KF_OK && res != KF_ENOCONV) return res;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (st) { st->iters = iters; st->rel_res_max = rm; }
  return res;
}

// ---------------------------------------------------------------------------
// KKT operator and preconditioner (eq. KKT, eq. precond, eq. precond_approx)
// ---------------------------------------------------------------------------
extern "C" kf_status kkt_apply(kf_problem *p, const void *xi, void *y) {
  CHECK_ST(check_p(p));
  if (!xi || !y) return fail(KF_EINVAL, "xi or y is NULL");
  if (xi == y) return fail(KF_EINVAL, "xi and y must not alias");
  if (!p->have_un) return fail(KF_ESTATE, "no background field (kf_set_background or newton_step first)");
  return launch_kkt_apply(p, (const double2 *)xi, (double2 *)y);
}

extern "C" kf_status kkt_apply_noalloc(kf_problem *p, const void *xi, void *y) {
  CHECK_ST(check_p(p));
  if (!xi || !y) return fail(KF_EINVAL, "xi or y is NULL");
  if (xi == y) return fail(KF_EINVAL, "xi and y must not alias");
  if (!p->have_un) return fail(KF_ESTATE, "no background field (kf_set_background or newton_step first)");
  return launch_kkt_apply_noalloc(p, (const double2 *)xi, (double2 *)y);
}

// ---------------------------------------------------------------------------
// L-BFGS H-block (Section 5: other approximations of H than L in the middle stage)
// ---------------------------------------------------------------------------
static kf_status read_c(kf_problem *p, const double2 *dev, double2 *host);

// z_s = Ht^-1 (y_s + P^* z_lam) by the two-loop recursion over the stored pairs with
// Ht0 = eps I, then z_u = y_lam + P z_s
static kf_status stage2_lbfgs(kf_problem *p, const double2 *y, double2 *z) {
  const size_t Ku = (size_t)p->K * p->Nu;
  const int64_t Ng = p->Ng;
  const double2 *ys = y + Ku, *yl = ys + Ng;
  double2 *zu = z, *zs = z + Ku;
  const double2 *zl = zs + Ng;
  double2 *q = p->hb_q, *dot = (double2 *)p->red_out;
  ProfScope ps(p, PROF_PRECOND);
  CHECK_ST(launch_gather_PH(p, 1.0, ys, 0.0, zl, 0, q));
  std::vector<double2> a(p->hb_n);
  for (int i = p->hb_n - 1; i >= 0; --i) {   // newest to oldest
    const int slot = ((p->hb_head - p->hb_n + i) % p->hb_max + p->hb_max) % p->hb_max;
    const double2 *si = p->hb_s + (size_t)slot * Ng, *yi = p->hb_y + (size_t)slot * Ng;
    double2 sq;
    CHECK_ST(dot_c128(p, si, q, Ng, dot));
    CHECK_ST(read_c(p, dot, &sq));
    a[i] = cscale(sq, p->hb_rho[slot]);
    CHECK_ST(launch_axpy_field(p, Ng, csub(make_double2(0.0, 0.0), a[i]), yi, q));
  }
  HIP_TRY(hipMemsetAsync(zs, 0, sizeof(double2) * Ng, p->stream));
  CHECK_ST(launch_axpy_field(p, Ng, make_double2(1.0 / p->eps, 0.0), q, zs));
  for (int i = 0; i < p->hb_n; ++i) {        // oldest to newest
    const int slot = ((p->hb_head - p->hb_n + i) % p->hb_max + p->hb_max) % p->hb_max;
    const double2 *si = p->hb_s + (size_t)slot * Ng, *yi = p->hb_y + (size_t)slot * Ng;
    double2 yr;
    CHECK_ST(dot_c128(p, yi, zs, Ng, dot));
    CHECK_ST(read_c(p, dot, &yr));
    const double2 b = cscale(yr, p->hb_rho[slot]);
    CHECK_ST(launch_axpy_field(p, Ng, csub(a[i], b), si, zs));
  }
  CHECK_ST(launch_scatter_P(p, zs, zu));
  return launch_axpy_field(p, (int64_t)Ku, make_double2(1.0, 0.0), yl, zu);
}

static kf_status hblock_add_pair(kf_problem *p, const double2 *s, const double2 *y) {
  const int64_t Ng = p->Ng;
  double ys = 0.0;
  {
    double2 c;
    CHECK_ST(dot_c128(p, y, s, Ng, (double2 *)p->red_out));
    CHECK_ST(read_c(p, (const double2 *)p->red_out, &c));
    ys = c.x;
  }
  if (!(ys > 0.0) || !std::isfinite(ys)) return fail(KF_EINVAL, "L-BFGS pair without positive curvature (Re y^H s <= 0)");
  const int slot = p->hb_head;
  HIP_TRY(hipMemcpyAsync(p->hb_s + (size_t)slot * Ng, s, sizeof(double2) * Ng, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->hb_y + (size_t)slot * Ng, y, sizeof(double2) * Ng, hipMemcpyDeviceToDevice, p->stream));
  p->hb_rho[slot] = 1.0 / ys;
  p->hb_head = (p->hb_head + 1) % p->hb_max;
  p->hb_n = std::min(p->hb_n + 1, p->hb_max);
  HIP_TRY(hipStreamSynchronize(p->stream));
  return KF_OK;
}

extern "C" kf_status kf_set_hblock(kf_problem *p, int32_t kind, int32_t max_pairs) {
  CHECK_ST(check_p(p));
  if (kind != KF_HBLOCK_EPS && kind != KF_HBLOCK_LBFGS) return fail(KF_EINVAL, "invalid H-block kind");
  if (kind == KF_HBLOCK_LBFGS && (max_pairs < 1 || max_pairs > 32)) return fail(KF_EINVAL, "max_pairs must be 1..32");
  HIP_TRY(hipStreamSynchronize(p->stream));
  dfree(p->hb_s); dfree(p->hb_y); dfree(p->hb_q);
  p->hb_n = p->hb_head = 0;
  p->hb_max = kind == KF_HBLOCK_LBFGS ? max_pairs : 0;
  p->hb_rho.assign((size_t)p->hb_max, 0.0);
  p->hblock = kind;
  if (kind == KF_HBLOCK_LBFGS) {
    CHECK_ST(dalloc(&p->hb_s, (size_t)max_pairs * p->Ng));
    CHECK_ST(dalloc(&p->hb_y, (size_t)max_pairs * p->Ng));
    CHECK_ST(dalloc(&p->hb_q, (size_t)p->Ng));
  }
  return KF_OK;
}

extern "C" kf_status kf_hblock_add_pair(kf_problem *p, const void *s, const void *y) {
  CHECK_ST(check_p(p));
  if (!s || !y) return fail(KF_EINVAL, "s or y is NULL");
  if (p->hblock != KF_HBLOCK_LBFGS) return fail(KF_ESTATE, "the H-block is not L-BFGS (kf_set_hblock first)");
  return hblock_add_pair(p, (const double2 *)s, (const double2 *)y);
}

// A~ of the multigrid variant: an inner iteration that stops at its tolerance or its
// iteration limit; the flexible outer Krylov method accepts either
static kf_status mg_inexact(kf_problem *p, int adjoint, const double2 *b, double2 *x) {
  kf_status st = mg_solve(p, adjoint, b, x, 0.0, 0, nullptr);
  return st == KF_ENOCONV ? KF_OK : st;
}

static kf_status precond_impl(kf_problem *p, int pc, const double2 *y, double2 *z) {
  const size_t Ku = (size_t)p->K * p->Nu;
  const double2 *yu = y;
  double2 *zu = z, *zl = z + Ku + p->Ng;
  // stage 1: z_lam = A^-* y_u
  if (pc == KF_PC_EXACT) CHECK_ST(blu_solve<double>(p, 1, yu, zl));
  else if (pc == KF_PC_INEXACT) CHECK_ST(blu_solve_mixed_io(p, 1, yu, zl));
  else CHECK_ST(mg_inexact(p, 1, yu, zl));
  // stage 2: z_s = Ht^-1 (y_s + P^* z_lam) (Ht = L = eps I, or L-BFGS), and z_u := y_lam + P z_s
  if (p->hblock == KF_HBLOCK_LBFGS && p->hb_n > 0) CHECK_ST(stage2_lbfgs(p, y, z));
  else CHECK_ST(launch_precond_stage2(p, y, z));
  // stage 3: z_u = A^-1 (y_lam + P z_s)
  if (pc == KF_PC_EXACT) CHECK_ST(blu_solve<double>(p, 0, zu, zu));
  else if (pc == KF_PC_INEXACT) CHECK_ST(blu_solve_mixed_io(p, 0, zu, zu));
  else CHECK_ST(mg_inexact(p, 0, zu, zu));
  return KF_OK;
}

// ---------------------------------------------------------------------------
// shifted-Laplacian multigrid (the inexact block solver of the third variant)
// ---------------------------------------------------------------------------
extern "C" kf_status kf_set_multigrid(kf_problem *p, int32_t prec, double beta, double inner_rtol, int32_t inner_maxit,
                                      int32_t n_min) {
  CHECK_ST(check_p(p));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return mg_configure(p, prec, beta, inner_rtol, inner_maxit, n_min);
}

extern "C" kf_status helmholtz_solve_mg(kf_problem *p, int32_t adjoint, const void *rhs, void *x, double rtol,
                                        int32_t maxit, kf_mg_stats *st) {
  CHECK_ST(check_p(p));
  if (!rhs || !x) return fail(KF_EINVAL, "rhs or x is NULL");
  if (!(rtol > 0.0 && rtol < 1.0) || maxit < 1) return fail(KF_EINVAL, "need 0 < rtol < 1 and maxit >= 1");
  kf_mg_stats S{};
  kf_status r = mg_solve(p, adjoint != 0, (const double2 *)rhs, (double2 *)x, rtol, maxit, &S);
  if (r != KF_OK && r != KF_ENOCONV) return r;
  // the true residual max_k ||rhs_k - op(A) x_k|| / ||rhs_k|| in FP64
  double rm = -1.0;
  if (rhs != x) CHECK_ST(residual_max(p, adjoint != 0, (const double2 *)rhs, (const double2 *)x, &rm, nullptr));
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.rel_res_max = rm;
  S.levels = mg_levels(p, nullptr);
  if (st) *st = S;
  return r;
}

extern "C" kf_status kf_mg_vcycle(kf_problem *p, const void *b, void *x) {
  CHECK_ST(check_p(p));
  if (!b || !x || b == x) return fail(KF_EINVAL, "b and x must be distinct non-NULL fields");
  return mg_vcycle_apply(p, (const double2 *)b, (double2 *)x);
}

extern "C" kf_status kf_mg_levels(kf_problem *p, int32_t *dims, int32_t *nlev) {
  CHECK_ST(check_p(p));
  if (!dims || !nlev) return fail(KF_EINVAL, "null pointer argument");
  int d[16] = {0};
  *nlev = mg_levels(p, d);
  for (int q = 0; q < 16; ++q) dims[q] = d[q];
  return KF_OK;
}

extern "C" kf_status precond_apply(kf_problem *p, int32_t pc, const void *y, void *z) {
  CHECK_ST(check_p(p));
  if (!y || !z) return fail(KF_EINVAL, "y or z is NULL");
  if (y == z) return fail(KF_EINVAL, "y and z must not alias");
  if (pc != KF_PC_EXACT && pc != KF_PC_INEXACT && pc != KF_PC_MULTIGRID) return fail(KF_EINVAL, "invalid preconditioner");
  if (!p->have_un) return fail(KF_ESTATE, "no background field (kf_set_background or newton_step first)");
  return precond_impl(p, pc, (const double2 *)y, (double2 *)z);
}

// ---------------------------------------------------------------------------
// flexible GMRES (right preconditioned, CGS2, Givens on the device)
// ---------------------------------------------------------------------------
// the packed right-hand side, solution and work vector of a KKT solve
static kf_status ensure_xi(kf_problem *p) {
  const size_t N = p->Nxi;
  if (!p->xi_w) CHECK_ST(dalloc(&p->xi_w, N));
  if (!p->xi_b) CHECK_ST(dalloc(&p->xi_b, N));
  if (!p->xi_x) CHECK_ST(dalloc(&p->xi_x, N));
  return KF_OK;
}

// the FGMRES(m) basis (m + 1 vectors), its preconditioned vectors (m) and Hessenberg data
static kf_status ensure_krylov(kf_problem *p, int m) {
  CHECK_ST(ensure_xi(p));
  if (p->krylov_m >= m) return KF_OK;
  dfree(p->V); dfree(p->Z); dfree(p->hess);
  p->krylov_m = 0;
  const size_t N = p->Nxi;
  CHECK_ST(dalloc(&p->V, (size_t)(m + 1) * N));
  CHECK_ST(dalloc(&p->Z, (size_t)m * N));
  CHECK_ST(dalloc(&p->hess, (size_t)(m + 1) * m + 6 * (size_t)(m + 1) + 16));
  p->krylov_m = m;
  return KF_OK;
}

struct FgmresOut {
  int iters = 0, restarts = 0, reorth = 0;
  double rel_res = 1.0;
  std::vector<double> hist;
  double ph[PH_N] = {0, 0, 0};
};

// Orthogonalise Vn = V_{j+1} against V_0..V_j in FP64 by classical Gram-Schmidt with
// selective reorthogonalisation, and normalise it.  The usual step is two sweeps over
// the basis: the dot products h1 = V^H Vn together with |Vn|^2, then the update
// Vn <- (Vn - V h1) / |Vn - V h1| with the norm taken from |Vn|^2 - |h1|^2 (V is
// orthonormal), decided on the device.  When the first pass cancels Vn below
// max(eta, 0.1) |Vn| the norm is measured by the update's sweep instead; below
// eta |Vn| a second pass (its dot products partly carried by the update's sweep, the
// rest, and the second update fused with the final norm) follows, then a scaling
// sweep.  Launches of a declined branch return at once, so the step needs no host
// round trip.  scal: [0] |Vn| after the last pass (the Hessenberg entry), [4] |Vn|^2
// before the first pass, [5] the first update's scale, [6] two int flags (second pass,
// measured norm).
static kf_status gram_schmidt(kf_problem *p, int j, double2 *Vn, double2 *h1, double2 *h2, double *scal,
                              double eta) {
  const int64_t N = p->Nxi;
  int *flags = (int *)(scal + 6);
  CHECK_ST(multidot_c128(p, p->V, j + 1, Vn, N, h1, nullptr, scal + 4));
  CHECK_ST(gs_decide(p, j + 1, h1, scal + 4, eta, h2, flags, scal + 0, scal + 5));
  CHECK_ST(axpy_dot_c128(p, p->V, j + 1, h1, Vn, N, h2, scal + 0, flags + 1, scal + 5, flags + 0));
  CHECK_ST(multidot_rest_c128(p, p->V, j + 1, Vn, N, h2, flags));
  CHECK_ST(axpy_dot_c128(p, p->V, j + 1, h2, Vn, N, nullptr, scal + 0, flags));
  CHECK_ST(scale_inv(p, N, scal + 0, Vn, Vn, flags + 1));
  return KF_OK;
}

static kf_status fgmres(kf_problem *p, int pc, const double2 *b, double2 *x, double tol, int m, int maxit, double eta,
                        FgmresOut &o) {
  const int64_t N = p->Nxi;
  double2 *H = p->hess;
  double2 *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *h1 = g + (m + 1), *h2 = h1 + (m + 1),
          *y = h2 + (m + 1);
  double *scal = (double *)(y + m + 8);  // [0] norm, [1] beta, [2] resid estimate, [3] ||b||
  PhaseTimer pt(p);
  CHECK_ST(norm_c128(p, b, N, scal + 3));
  HIP_TRY(hipMemcpyAsync(p->host_pinned, scal + 3, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const double bnorm = p->host_pinned[0];
  HIP_TRY(hipMemsetAsync(x, 0, sizeof(double2) * N, p->stream));
  o.hist.assign(1, 1.0);
  if (!std::isfinite(bnorm)) return fail(KF_ENAN, "non-finite right-hand side");
  if (bnorm == 0.0) { o.rel_res = 0.0; return KF_OK; }
  int total = 0;
  kf_status status = KF_OK;
  for (;;) {
    double2 *V0 = p->V;
    if (total == 0) {
      HIP_TRY(hipMemcpyAsync(V0, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
    } else {
      pt.start(PH_MATVEC);
      CHECK_ST(launch_kkt_apply(p, x, p->xi_w));
      pt.stop();
      HIP_TRY(hipMemcpyAsync(V0, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
      CHECK_ST(launch_axpy_field(p, N, make_double2(-1.0, 0.0), p->xi_w, V0));
    }
    CHECK_ST(norm_c128(p, V0, N, scal + 1));
    HIP_TRY(hipMemcpyAsync(p->host_pinned, scal + 1, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    const double beta = p->host_pinned[0];
    if (!std::isfinite(beta)) { status = fail(KF_ENAN, "non-finite residual in FGMRES"); break; }
    o.rel_res = beta / bnorm;
    if (o.rel_res <= tol) break;
    if (total >= maxit) { status = fail(KF_ENOCONV, "FGMRES reached maxit"); break; }
    CHECK_ST(scale_inv(p, N, scal + 1, V0, V0));
    CHECK_ST(set_g0(p, m, scal + 1, g));
    int nj = 0;
    bool breakdown = false;
    for (int j = 0; j < m; ++j) {
      double2 *Vj = p->V + (size_t)j * N, *Vn = p->V + (size_t)(j + 1) * N, *Zj = p->Z + (size_t)j * N;
      pt.start(PH_PRECOND);
      CHECK_ST(precond_impl(p, pc, Vj, Zj));
      pt.stop();
      pt.start(PH_MATVEC);
      CHECK_ST(launch_kkt_apply(p, Zj, Vn));
      pt.stop();
      pt.start(PH_ORTH);
      CHECK_ST(gram_schmidt(p, j, Vn, h1, h2, scal, eta));
      CHECK_ST(arnoldi_finish(p, j, m, h1, h2, scal + 0, H, cs, sn, g, scal + 2));
      pt.stop();
      HIP_TRY(hipMemcpyAsync(p->host_pinned, scal, 7 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      const double hn = p->host_pinned[0], est = p->host_pinned[2] / bnorm;
      o.reorth += *(const int *)(p->host_pinned + 6);
      ++total;
      nj = j + 1;
      o.hist.push_back(est);
      if (!std::isfinite(est) || !std::isfinite(hn)) { status = fail(KF_ENAN, "non-finite value in Arnoldi"); break; }
      if (hn == 0.0) { breakdown = true; break; }   // exact solution in the current space
      if (est <= tol || total >= maxit) break;
    }
    if (status != KF_OK) break;
    pt.start(PH_ORTH);
    CHECK_ST(hess_backsolve(p, nj, m, H, g, y));
    CHECK_ST(multiaxpy_c128(p, p->Z, nj, y, 1.0, x, N));
    pt.stop();
    o.restarts += 1;
    (void)breakdown;
  }
  o.iters = total;
  pt.sum(o.ph, PH_N);
  return status;
}

// ---------------------------------------------------------------------------
// outer BiCGStab (the Conclusions' memory-lean alternative to GMRES): right-
// preconditioned, nine packed vectors whatever the iteration count
// ---------------------------------------------------------------------------
static double host_norm(kf_problem *p, const double2 *x, int64_t n, kf_status *st);
static kf_status hessian_apply(kf_problem *p, const kf_cg_opts *o, const double2 *v, double2 *out, int *solves);

static kf_status read_c(kf_problem *p, const double2 *dev, double2 *host) {
  HIP_TRY(hipMemcpyAsync(p->host_pinned, dev, sizeof(double2), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  host->x = p->host_pinned[0];
  host->y = p->host_pinned[1];
  return KF_OK;
}

static inline double2 cdiv_h(double2 a, double2 b) { return cdiv(a, b); }

static kf_status bicgstab_outer(kf_problem *p, int pc, const double2 *b, double2 *x, double tol, int maxit,
                                FgmresOut &o) {
  const int64_t N = p->Nxi;
  if (!p->bicg) CHECK_ST(dalloc(&p->bicg, (size_t)8 * N));
  double2 *r = p->bicg, *rh = r + N, *pv = rh + N, *v = pv + N, *sv = v + N, *t = sv + N, *ph = t + N, *sh = ph + N;
  double2 *dot = (double2 *)p->red_out;
  PhaseTimer pt(p);
  kf_status e = KF_OK;
  const double bnorm = host_norm(p, b, N, &e);
  CHECK_ST(e);
  HIP_TRY(hipMemsetAsync(x, 0, sizeof(double2) * N, p->stream));
  o.hist.assign(1, 1.0);
  if (!std::isfinite(bnorm)) return fail(KF_ENAN, "non-finite right-hand side");
  if (bnorm == 0.0) { o.rel_res = 0.0; return KF_OK; }
  HIP_TRY(hipMemcpyAsync(r, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(rh, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemsetAsync(pv, 0, sizeof(double2) * N, p->stream));
  HIP_TRY(hipMemsetAsync(v, 0, sizeof(double2) * N, p->stream));
  double2 rho = make_double2(1.0, 0.0), alpha = rho, omega = rho;
  const double2 one = make_double2(1.0, 0.0);
  kf_status status = KF_OK;
  int it = 0;
  double rel = 1.0;
  for (;;) {
    if (it >= maxit) { status = fail(KF_ENOCONV, "outer BiCGStab reached maxit"); break; }
    double2 rho_new;
    pt.start(PH_ORTH);
    CHECK_ST(dot_c128(p, rh, r, N, dot));
    CHECK_ST(read_c(p, dot, &rho_new));
    if (cabs2(rho_new) == 0.0 || cabs2(omega) == 0.0) { status = fail(KF_EBREAKDOWN, "outer BiCGStab breakdown"); break; }
    const double2 beta = cmul(cdiv_h(rho_new, rho), cdiv_h(alpha, omega));
    // p = r + beta (p - omega v)
    CHECK_ST(launch_axpy_field(p, N, csub(make_double2(0.0, 0.0), omega), v, pv));
    CHECK_ST(launch_axpby_field(p, N, one, r, beta, pv));
    pt.stop();
    pt.start(PH_PRECOND);
    CHECK_ST(precond_impl(p, pc, pv, ph));
    pt.stop();
    pt.start(PH_MATVEC);
    CHECK_ST(launch_kkt_apply(p, ph, v));
    pt.stop();
    pt.start(PH_ORTH);
    double2 rv;
    CHECK_ST(dot_c128(p, rh, v, N, dot));
    CHECK_ST(read_c(p, dot, &rv));
    if (cabs2(rv) == 0.0) { status = fail(KF_EBREAKDOWN, "outer BiCGStab breakdown"); pt.stop(); break; }
    alpha = cdiv_h(rho_new, rv);
    // s = r - alpha v
    HIP_TRY(hipMemcpyAsync(sv, r, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
    CHECK_ST(launch_axpy_field(p, N, csub(make_double2(0.0, 0.0), alpha), v, sv));
    pt.stop();
    pt.start(PH_PRECOND);
    CHECK_ST(precond_impl(p, pc, sv, sh));
    pt.stop();
    pt.start(PH_MATVEC);
    CHECK_ST(launch_kkt_apply(p, sh, t));
    pt.stop();
    pt.start(PH_ORTH);
    double2 ts, tt;
    CHECK_ST(dot_c128(p, t, sv, N, dot));
    CHECK_ST(read_c(p, dot, &ts));
    CHECK_ST(dot_c128(p, t, t, N, dot));
    CHECK_ST(read_c(p, dot, &tt));
    omega = tt.x > 0.0 ? cdiv_h(ts, tt) : make_double2(0.0, 0.0);
    // x += alpha ph + omega sh;  r = s - omega t
    CHECK_ST(launch_axpy_field(p, N, alpha, ph, x));
    CHECK_ST(launch_axpy_field(p, N, omega, sh, x));
    CHECK_ST(launch_axpby_field(p, N, csub(make_double2(0.0, 0.0), omega), t, one, sv));
    HIP_TRY(hipMemcpyAsync(r, sv, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
    rho = rho_new;
    const double rn = host_norm(p, r, N, &e);
    CHECK_ST(e);
    pt.stop();
    ++it;
    rel = rn / bnorm;
    o.hist.push_back(rel);
    if (!std::isfinite(rel)) { status = fail(KF_ENAN, "non-finite residual in outer BiCGStab"); break; }
    if (rel <= tol) {
      // the true residual decides: b - M x
      CHECK_ST(launch_kkt_apply(p, x, p->xi_w));
      HIP_TRY(hipMemcpyAsync(t, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
      CHECK_ST(launch_axpy_field(p, N, make_double2(-1.0, 0.0), p->xi_w, t));
      const double tn = host_norm(p, t, N, &e);
      CHECK_ST(e);
      rel = tn / bnorm;
      if (rel <= tol) break;
      // the recurrence drifted: restart from the true residual
      HIP_TRY(hipMemcpyAsync(r, t, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
      HIP_TRY(hipMemcpyAsync(rh, t, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
      HIP_TRY(hipMemsetAsync(pv, 0, sizeof(double2) * N, p->stream));
      HIP_TRY(hipMemsetAsync(v, 0, sizeof(double2) * N, p->stream));
      rho = alpha = omega = one;
    }
  }
  o.iters = it;
  o.rel_res = rel;
  pt.sum(o.ph, PH_N);
  return status;
}

// ---------------------------------------------------------------------------
// one Gauss-Newton step in the full space (Sections 3-5)
// ---------------------------------------------------------------------------
static double host_norm(kf_problem *p, const double2 *x, int64_t n, kf_status *st) {
  *st = norm_c128(p, x, n, p->red_out);
  if (*st != KF_OK) return NAN;
  if (hipMemcpyAsync(p->host_pinned, p->red_out, sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    *st = fail(KF_EHIP, "readback failed");
    return NAN;
  }
  return p->host_pinned[0];
}

static kf_status forward_solve(kf_problem *p, int prec, double rtol, double2 *u, int *iters) {
  CHECK_ST(launch_sources(p, p->vec_c));
  *iters = 1;
  if (prec == KF_MIXED) {
    double rm;
    kf_status st = solve_mixed(p, 0, p->vec_c, u, rtol, 20, iters, &rm);
    return st;
  }
  return blu_solve<double>(p, 0, p->vec_c, u);
}

extern "C" kf_status newton_step(kf_problem *p, const void *d_obs, const kf_newton_opts *o, void *xi_out,
                                 double *gamma_next, int32_t update_in_place, kf_newton_stats *st) {
  CHECK_ST(check_p(p));
  if (!d_obs || !o) return fail(KF_EINVAL, "d_obs or opts is NULL");
  if (!(o->rtol > 0.0) || o->restart < 1 || o->restart > 200 || o->maxit < 1)
    return fail(KF_EINVAL, "need rtol > 0, 1 <= restart <= 200, maxit >= 1");
  if (o->pc != KF_PC_EXACT && o->pc != KF_PC_INEXACT && o->pc != KF_PC_MULTIGRID)
    return fail(KF_EINVAL, "invalid preconditioner");
  if (o->fwd_prec != KF_C128 && o->fwd_prec != KF_MIXED) return fail(KF_EINVAL, "fwd_prec must be C128 or MIXED");
  if (o->fwd_prec == KF_MIXED && !(o->fwd_rtol > 0.0)) return fail(KF_EINVAL, "fwd_rtol must be > 0");
  if (!(o->reorth_eta >= 0.0 && o->reorth_eta <= 1.0)) return fail(KF_EINVAL, "reorth_eta must be in [0, 1]");
  if (o->outer != KF_OUTER_FGMRES && o->outer != KF_OUTER_BICGSTAB) return fail(KF_EINVAL, "invalid outer solver");
  kf_newton_stats S;
  std::memset(&S, 0, sizeof(S));
  S.misfit_after = -1.0;
  auto T0 = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  if (o->outer == KF_OUTER_BICGSTAB) CHECK_ST(ensure_xi(p));
  else CHECK_ST(ensure_krylov(p, o->restart));
  const int64_t N = p->Nxi;
  const size_t Ku = (size_t)p->K * p->Nu;
  // factorisation of A(gamma_n)
  HIP_TRY(hipStreamSynchronize(p->stream));
  auto t = std::chrono::steady_clock::now();
  int which = 1 | ((o->pc == KF_PC_INEXACT || o->fwd_prec == KF_MIXED) ? 2 : 0);
  CHECK_ST(blu_factor(p, which));
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_factor_ms = ms_since(t);
  // background field u_n = A^-1 f
  t = std::chrono::steady_clock::now();
  int fit = 0;
  CHECK_ST(forward_solve(p, o->fwd_prec, o->fwd_rtol, p->u_n, &fit));
  p->have_un = true;
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_forward_ms = ms_since(t);
  S.fwd_refine_iters = fit;
  // data residual and right-hand side b (eq. KKT)
  kf_status e = KF_OK;
  CHECK_ST(launch_residual(p, (const double2 *)d_obs, p->u_n, p->d_r, p->d_wr));
  const int64_t nd = (int64_t)p->K * p->nrec;
  double rn = host_norm(p, p->d_r, nd, &e); CHECK_ST(e);
  double dn = host_norm(p, (const double2 *)d_obs, nd, &e); CHECK_ST(e);
  double wn = host_norm(p, p->d_wr, nd, &e); CHECK_ST(e);
  S.misfit_before = dn > 0 ? rn / dn : rn;
  S.phi_before = 0.5 * wn * wn;
  CHECK_ST(launch_rhs(p, p->d_r, p->d_rptr, p->d_rlist, p->xi_b, p->d.reg_on_update));
  // KKT solve
  FgmresOut fo;
  kf_status fst = o->outer == KF_OUTER_BICGSTAB
                      ? bicgstab_outer(p, o->pc, p->xi_b, p->xi_x, o->rtol, o->maxit, fo)
                      : fgmres(p, o->pc, p->xi_b, p->xi_x, o->rtol, o->restart, o->maxit, o->reorth_eta, fo);
  if (fst != KF_OK && fst != KF_ENOCONV) return fst;
  S.outer_iters = fo.iters;
  S.reorth_passes = fo.reorth;
  S.restarts = fo.restarts;
  S.rel_res = fo.rel_res;
  for (size_t q = 1; q < fo.hist.size() && q <= 512; ++q) S.rel_res_hist[q - 1] = fo.hist[q];
  S.t_precond_ms = fo.ph[PH_PRECOND];
  S.t_matvec_ms = fo.ph[PH_MATVEC];
  S.t_orth_ms = fo.ph[PH_ORTH];
  // ||Im ds|| / ||ds||
  const double2 *ds = p->xi_x + Ku;
  double dsn = host_norm(p, ds, p->Ng, &e); CHECK_ST(e);
  CHECK_ST(imag_part(p, p->Ng, ds, p->vec_a));
  double dsi = host_norm(p, p->vec_a, p->Ng, &e); CHECK_ST(e);
  S.ds_imag_ratio = dsn > 0 ? dsi / dsn : 0.0;
  if (xi_out) HIP_TRY(hipMemcpyAsync(xi_out, p->xi_x, sizeof(double2) * N, hipMemcpyDeviceToDevice, p->stream));
  // L-BFGS H-block: the step gives the pair (ds, H ds) at gamma_n for the next steps
  if (p->hblock == KF_HBLOCK_LBFGS && fst == KF_OK) {
    if (!p->cg_vec) CHECK_ST(dalloc(&p->cg_vec, (size_t)5 * p->Ng));
    if (!p->cg_field) CHECK_ST(dalloc(&p->cg_field, (size_t)p->K * p->Nu));
    kf_cg_opts ho{};
    ho.solve_prec = KF_C128;
    int solves = 0;
    CHECK_ST(hessian_apply(p, &ho, ds, p->cg_vec, &solves));
    kf_status hs = hblock_add_pair(p, ds, p->cg_vec);
    if (hs != KF_OK && hs != KF_EINVAL) return hs;   // a pair without curvature is skipped
  }
  // gamma_{n+1} = gamma_n + Re(ds) on the core
  if (update_in_place || o->misfit_after) {
    if (!update_in_place) HIP_TRY(hipMemcpyAsync(p->vec_d, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
    CHECK_ST(launch_update_gamma(p, ds, p->gamma));
    p->have_T64 = p->have_T32 = false;
    ++p->gamma_version;
    if (gamma_next) HIP_TRY(hipMemcpyAsync(gamma_next, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
    if (o->misfit_after) {
      CHECK_ST(blu_factor(p, o->fwd_prec == KF_MIXED ? 3 : 1));
      int it2;
      // the outer solver's vectors are free after the solve: at least 2 packed vectors > K*Nu
      double2 *u1 = o->outer == KF_OUTER_BICGSTAB ? p->bicg : p->V;
      CHECK_ST(forward_solve(p, o->fwd_prec, o->fwd_rtol, u1, &it2));
      CHECK_ST(launch_residual(p, (const double2 *)d_obs, u1, p->d_r, p->d_wr));
      double rn1 = host_norm(p, p->d_r, nd, &e); CHECK_ST(e);
      S.misfit_after = dn > 0 ? rn1 / dn : rn1;
    }
    if (!update_in_place) {
      // restore gamma_n (kept in vec_d, which no step above overwrote)
      HIP_TRY(hipMemcpyAsync(p->gamma, p->vec_d, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
      p->have_T64 = p->have_T32 = false;
      ++p->gamma_version;
    }
  } else if (gamma_next) {
    HIP_TRY(hipMemcpyAsync(gamma_next, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
    CHECK_ST(launch_update_gamma(p, ds, gamma_next));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_total_ms = ms_since(T0);
  if (st) *st = S;
  prof_collect(p);
  return fst;
}

// ---------------------------------------------------------------------------
// independent problems stepped at once, each on a stream and a host thread of its own
// ---------------------------------------------------------------------------
constexpr int KF_CONCURRENT_MAX = 16;
extern "C" kf_status newton_step_concurrent(kf_problem *const *problems, int32_t n, const void *const *d_obs,
                                            const kf_newton_opts *opts, void *const *xi_out,
                                            double *const *gamma_next, int32_t update_in_place,
                                            kf_newton_stats *st) {
  if (!problems || !d_obs || !opts) return fail(KF_EINVAL, "null pointer argument");
  if (n < 1 || n > KF_CONCURRENT_MAX) return fail(KF_EINVAL, "need 1..16 problems");
  for (int q = 0; q < n; ++q) {
    if (!problems[q] || !d_obs[q]) return fail(KF_EINVAL, "problem or data " + std::to_string(q) + " is NULL");
    for (int r = 0; r < q; ++r)
      if (problems[r] == problems[q]) return fail(KF_EINVAL, "problem " + std::to_string(q) + " appears twice");
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::vector<hipStream_t> saved(n), own(n, nullptr);
  for (int q = 0; q < n; ++q) {
    saved[q] = problems[q]->stream;
    HIP_TRY(hipStreamSynchronize(saved[q]));   // the caller's work on this problem is done
  }
  for (int q = 0; q < n; ++q) {
    const hipError_t e = hipStreamCreateWithFlags(&own[q], hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int r = 0; r < q; ++r) hipStreamDestroy(own[r]);
      return fail(KF_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
    }
  }
  for (int q = 0; q < n; ++q) problems[q]->stream = own[q];
  std::vector<kf_status> rs(n, KF_OK);
  std::vector<std::string> msg(n);
  std::vector<kf_newton_stats> S(n);
  {
    std::vector<std::thread> workers;
    workers.reserve(n);
    for (int q = 0; q < n; ++q)
      workers.emplace_back([&, q] {
        // the device is per host thread; the error text of newton_step is this thread's
        if (hipSetDevice(dev) != hipSuccess) {
          rs[q] = KF_EHIP;
          msg[q] = "hipSetDevice failed in a worker thread";
          return;
        }
        rs[q] = newton_step(problems[q], d_obs[q], opts, xi_out ? xi_out[q] : nullptr,
                            gamma_next ? gamma_next[q] : nullptr, update_in_place, &S[q]);
        if (rs[q] != KF_OK) msg[q] = g_last_error;
        hipStreamSynchronize(own[q]);
      });
    for (auto &w : workers) w.join();
  }
  for (int q = 0; q < n; ++q) {
    problems[q]->stream = saved[q];
    hipStreamDestroy(own[q]);
  }
  if (st)
    for (int q = 0; q < n; ++q) st[q] = S[q];
  int bad = -1;
  for (int q = 0; q < n && bad < 0; ++q)
    if (rs[q] != KF_OK && rs[q] != KF_ENOCONV) bad = q;
  for (int q = 0; q < n && bad < 0; ++q)
    if (rs[q] == KF_ENOCONV) bad = q;
  if (bad < 0) return KF_OK;
  return fail(rs[bad], "problem " + std::to_string(bad) + ": " + msg[bad]);
}

// ---------------------------------------------------------------------------
// frequency continuation (Section 6, the frequency sweep)
// ---------------------------------------------------------------------------
extern "C" kf_status newton_continuation(kf_problem *const *problems, int32_t n, const void *const *d_obs,
                                         const int32_t *steps, const kf_newton_opts *opts, double *gamma_out,
                                         kf_newton_stats *st) {
  if (!problems || !d_obs || !steps || !opts) return fail(KF_EINVAL, "null pointer argument");
  if (n < 1) return fail(KF_EINVAL, "need at least one problem");
  for (int q = 0; q < n; ++q) {
    if (!problems[q] || !d_obs[q]) return fail(KF_EINVAL, "problem or data " + std::to_string(q) + " is NULL");
    if (steps[q] < 0) return fail(KF_EINVAL, "steps must be >= 0");
    const kf_problem *a = problems[0], *b = problems[q];
    if (a->nx != b->nx || a->nz != b->nz || a->npml != b->npml || a->h != b->h)
      return fail(KF_ESHAPE, "continuation problems must share the grid (nx, nz, h, npml)");
  }
  int i = 0;
  for (int q = 0; q < n; ++q) {
    kf_problem *p = problems[q];
    if (q > 0) {   // the previous frequency's model starts this one
      HIP_TRY(hipStreamSynchronize(problems[q - 1]->stream));
      CHECK_ST(kf_set_gamma(p, problems[q - 1]->gamma));
    }
    for (int s = 0; s < steps[q]; ++s) {
      kf_newton_stats S;
      kf_status r = newton_step(p, d_obs[q], opts, nullptr, nullptr, 1, &S);
      if (st) st[i] = S;
      ++i;
      if (r != KF_OK) return r;
    }
  }
  kf_problem *last = problems[n - 1];
  if (gamma_out) HIP_TRY(hipMemcpyAsync(gamma_out, last->gamma, sizeof(double) * last->Nu, hipMemcpyDeviceToDevice,
                                        last->stream));
  HIP_TRY(hipStreamSynchronize(last->stream));
  return KF_OK;
}

// ---------------------------------------------------------------------------
// reduced-space Gauss-Newton step by conjugate gradients (Section 3; Table 1 "CG")
// ---------------------------------------------------------------------------
static kf_status cg_solve_field(kf_problem *p, int adjoint, int prec, double rtol, const double2 *rhs, double2 *x,
                                int *solves) {
  *solves += 1;
  if (prec == KF_MIXED) {
    int it = 0;
    double rm = 0.0;
    return solve_mixed(p, adjoint, rhs, x, rtol, 30, &it, &rm);
  }
  return blu_solve<double>(p, adjoint, rhs, x);
}

// out = H v (real part only when real_only), by one forward and one adjoint block solve
// of all sources; uses vec_d and cg_field
static kf_status hessian_apply(kf_problem *p, const kf_cg_opts *o, const double2 *v, double2 *out, int *solves) {
  CHECK_ST(launch_scatter_P(p, v, p->vec_d));
  CHECK_ST(cg_solve_field(p, 0, o->solve_prec, o->solve_rtol, p->vec_d, p->cg_field, solves));
  CHECK_ST(launch_apply_F(p, p->cg_field, p->vec_d));
  CHECK_ST(cg_solve_field(p, 1, o->solve_prec, o->solve_rtol, p->vec_d, p->cg_field, solves));
  return launch_gather_PH(p, p->eps, v, 0.0, p->cg_field, o->real_constrained, out);
}

static kf_status read_scalar(kf_problem *p, const double *dev, double *host) {
  HIP_TRY(hipMemcpyAsync(p->host_pinned, dev, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *host = p->host_pinned[0];
  return KF_OK;
}

// Re(a^H b) read back to the host
static kf_status host_dot_re(kf_problem *p, const double2 *a, const double2 *b, int64_t n, double *out) {
  CHECK_ST(dot_c128(p, a, b, n, (double2 *)p->red_out));
  return read_scalar(p, p->red_out, out);
}

extern "C" kf_status rsgn_cg_step(kf_problem *p, const void *d_obs, const kf_cg_opts *o, void *ds_out,
                                  double *gamma_next, int32_t update_in_place, kf_cg_stats *st) {
  CHECK_ST(check_p(p));
  if (!d_obs || !o) return fail(KF_EINVAL, "d_obs or opts is NULL");
  if (!(o->rtol > 0.0) || o->maxit < 1) return fail(KF_EINVAL, "need rtol > 0 and maxit >= 1");
  if (o->solve_prec != KF_C128 && o->solve_prec != KF_MIXED) return fail(KF_EINVAL, "solve_prec must be C128 or MIXED");
  if (o->solve_prec == KF_MIXED && !(o->solve_rtol > 0.0)) return fail(KF_EINVAL, "solve_rtol must be > 0");
  if (o->fwd_prec != KF_C128 && o->fwd_prec != KF_MIXED) return fail(KF_EINVAL, "fwd_prec must be C128 or MIXED");
  if (o->fwd_prec == KF_MIXED && !(o->fwd_rtol > 0.0)) return fail(KF_EINVAL, "fwd_rtol must be > 0");
  kf_cg_stats S;
  std::memset(&S, 0, sizeof(S));
  auto T0 = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  const int64_t Ng = p->Ng;
  if (!p->cg_vec) CHECK_ST(dalloc(&p->cg_vec, (size_t)5 * Ng));
  if (!p->cg_field) CHECK_ST(dalloc(&p->cg_field, (size_t)p->K * p->Nu));
  double2 *x = p->cg_vec, *r = x + Ng, *d = r + Ng, *Hd = d + Ng, *g = Hd + Ng;
  // factorisation and background field u_n = A^-1 f
  HIP_TRY(hipStreamSynchronize(p->stream));
  auto t = std::chrono::steady_clock::now();
  const bool need32 = o->fwd_prec == KF_MIXED || o->solve_prec == KF_MIXED;
  CHECK_ST(blu_factor(p, 1 | (need32 ? 2 : 0)));
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_factor_ms = ms_since(t);
  t = std::chrono::steady_clock::now();
  int fit = 0;
  CHECK_ST(forward_solve(p, o->fwd_prec, o->fwd_rtol, p->u_n, &fit));
  p->have_un = true;
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_forward_ms = ms_since(t);
  // data residual, misfit and the gradient g = sum_k J_k^* W_k^2 r_k (- eps s_n)
  kf_status e = KF_OK;
  CHECK_ST(launch_residual(p, (const double2 *)d_obs, p->u_n, p->d_r, p->d_wr));
  const int64_t nd = (int64_t)p->K * p->nrec;
  double rn = host_norm(p, p->d_r, nd, &e); CHECK_ST(e);
  double dn = host_norm(p, (const double2 *)d_obs, nd, &e); CHECK_ST(e);
  double wn = host_norm(p, p->d_wr, nd, &e); CHECK_ST(e);
  S.misfit_before = dn > 0 ? rn / dn : rn;
  S.phi_before = 0.5 * wn * wn;
  t = std::chrono::steady_clock::now();
  int solves = 0;
  CHECK_ST(launch_rhs_u_field(p, p->d_r, p->vec_d));
  CHECK_ST(cg_solve_field(p, 1, o->solve_prec, o->solve_rtol, p->vec_d, p->cg_field, &solves));
  CHECK_ST(launch_gather_PH(p, 0.0, nullptr, p->d.reg_on_update ? 0.0 : -p->eps, p->cg_field, o->real_constrained, g));
  // CG on H ds = g from ds = 0
  HIP_TRY(hipMemsetAsync(x, 0, sizeof(double2) * Ng, p->stream));
  HIP_TRY(hipMemcpyAsync(r, g, sizeof(double2) * Ng, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(d, g, sizeof(double2) * Ng, hipMemcpyDeviceToDevice, p->stream));
  double rr = 0.0;
  CHECK_ST(host_dot_re(p, r, r, Ng, &rr));
  const double gn = std::sqrt(rr);
  if (!std::isfinite(gn)) return fail(KF_ENAN, "non-finite gradient");
  kf_status status = KF_OK;
  int it = 0;
  double rel = gn > 0.0 ? 1.0 : 0.0;
  while (gn > 0.0 && rel > o->rtol) {
    if (it >= o->maxit) { status = fail(KF_ENOCONV, "RSGN-CG reached maxit"); break; }
    CHECK_ST(hessian_apply(p, o, d, Hd, &solves));
    double dHd = 0.0;
    CHECK_ST(host_dot_re(p, d, Hd, Ng, &dHd));
    if (!(dHd > 0.0)) { status = fail(dHd == dHd ? KF_EBREAKDOWN : KF_ENAN, "RSGN-CG: d^H H d is not positive"); break; }
    const double alpha = rr / dHd;
    CHECK_ST(launch_axpy_field(p, Ng, make_double2(alpha, 0.0), d, x));
    CHECK_ST(launch_axpy_field(p, Ng, make_double2(-alpha, 0.0), Hd, r));
    double rr_new = 0.0;
    CHECK_ST(host_dot_re(p, r, r, Ng, &rr_new));
    if (!std::isfinite(rr_new)) { status = fail(KF_ENAN, "non-finite CG residual"); break; }
    CHECK_ST(launch_axpby_field(p, Ng, make_double2(1.0, 0.0), r, make_double2(rr_new / rr, 0.0), d));
    rr = rr_new;
    ++it;
    rel = std::sqrt(rr) / gn;
    if (it <= 512) S.rel_res_hist[it - 1] = rel;
  }
  S.iters = it;
  S.rel_res = rel;
  // the true E_cg = ||H ds - g|| / ||g|| at exit (one more Hessian product)
  if (status == KF_OK && gn > 0.0) {
    CHECK_ST(hessian_apply(p, o, x, Hd, &solves));
    CHECK_ST(launch_axpy_field(p, Ng, make_double2(-1.0, 0.0), g, Hd));
    double t2 = 0.0;
    CHECK_ST(host_dot_re(p, Hd, Hd, Ng, &t2));
    S.true_rel_res = std::sqrt(t2) / gn;
  }
  S.solves = solves;
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_cg_ms = ms_since(t);
  if (ds_out) HIP_TRY(hipMemcpyAsync(ds_out, x, sizeof(double2) * Ng, hipMemcpyDeviceToDevice, p->stream));
  if (update_in_place) {
    CHECK_ST(launch_update_gamma(p, x, p->gamma));
    p->have_T64 = p->have_T32 = false;
    ++p->gamma_version;
    p->have_un = false;
    if (gamma_next) HIP_TRY(hipMemcpyAsync(gamma_next, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
  } else if (gamma_next) {
    HIP_TRY(hipMemcpyAsync(gamma_next, p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, p->stream));
    CHECK_ST(launch_update_gamma(p, x, gamma_next));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  S.t_total_ms = ms_since(T0);
  if (st) *st = S;
  return status;
}

// ---------------------------------------------------------------------------
// reduced gradient through the forward solve (autograd backward)
// ---------------------------------------------------------------------------
extern "C" kf_status helmholtz_adjoint_gradient(kf_problem *p, int32_t prec, const void *u, const void *grad_u,
                                                double *grad_gamma) {
  CHECK_ST(check_p(p));
  if (!u || !grad_u || !grad_gamma) return fail(KF_EINVAL, "null pointer argument");
  if (prec == KF_C128) {
    CHECK_ST(blu_solve<double>(p, 1, (const double2 *)grad_u, p->vec_a));
    CHECK_ST(launch_grad_gamma(p, u, p->vec_a, 0, grad_gamma));
  } else if (prec == KF_C64) {
    float2 *mu = (float2 *)p->vec_a;
    CHECK_ST(blu_solve<float>(p, 1, (const float2 *)grad_u, mu));
    CHECK_ST(launch_grad_gamma(p, u, mu, 1, grad_gamma));
  } else if (prec == KF_MIXED) {
    int it;
    double rm;
    CHECK_ST(solve_mixed(p, 1, (const double2 *)grad_u, p->vec_d, 1e-12, 10, &it, &rm));
    CHECK_ST(launch_grad_gamma(p, u, p->vec_d, 0, grad_gamma));
  } else {
    return fail(KF_EINVAL, "invalid precision");
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return KF_OK;
}

// ---------------------------------------------------------------------------
// profiling API
// ---------------------------------------------------------------------------
static const char *prof_names[PROF_N] = {"kkt_apply", "stencil",     "blu_factor",  "blu_sweep",
                                         "precond_stage", "orth",  "reduce",      "blu_fwd_c128",
                                         "blu_fwd_c64",   "blu_bwd_c128", "blu_bwd_c64", "blu_mid",
                                         "blu_reduced_rhs", "blu_chain", "blu_correct", "gs_dot",
                                         "gs_update", "mg_solve"};

extern "C" kf_status kf_profile_enable(kf_problem *p, int32_t on) {
  CHECK_ST(check_p(p));
  prof_collect(p);
  p->prof = on != 0;
  for (int i = 0; i < PROF_N; ++i) p->counters[i] = ProfCounter();
  return KF_OK;
}

extern "C" kf_status kf_profile_only(kf_problem *p, const char *name) {
  CHECK_ST(check_p(p));
  prof_collect(p);
  if (!name || !*name) {
    p->prof_mask = ~0u;
    return KF_OK;
  }
  for (int i = 0; i < PROF_N; ++i)
    if (std::strcmp(name, prof_names[i]) == 0) {
      p->prof_mask = 1u << i;
      return KF_OK;
    }
  return fail(KF_EINVAL, std::string("unknown kernel family ") + name);
}

extern "C" kf_status kf_profile_work(kf_problem *p, const char *name, double *work) {
  CHECK_ST(check_p(p));
  if (!name || !work) return fail(KF_EINVAL, "null pointer argument");
  prof_collect(p);
  for (int i = 0; i < PROF_N; ++i)
    if (std::strcmp(name, prof_names[i]) == 0) {
      *work = p->counters[i].work;
      return KF_OK;
    }
  return fail(KF_EINVAL, std::string("unknown kernel family ") + name);
}

extern "C" kf_status kf_profile_read(kf_problem *p, const char *name, int64_t *launches, double *total_ms) {
  CHECK_ST(check_p(p));
  if (!name || !launches || !total_ms) return fail(KF_EINVAL, "null pointer argument");
  prof_collect(p);
  for (int i = 0; i < PROF_N; ++i)
    if (std::strcmp(name, prof_names[i]) == 0) {
      *launches = p->counters[i].launches;
      *total_ms = p->counters[i].ms;
      return KF_OK;
    }
  return fail(KF_EINVAL, std::string("unknown kernel family ") + name);
}

// ---------------------------------------------------------------------------
// batches: several problems (frequencies, uneven grids) advanced together
// ---------------------------------------------------------------------------
struct kf_batch {
  std::vector<kf_problem *> p;
  std::vector<hipStream_t> prev_stream;  // each problem's stream before it joined the batch
  hipStream_t stream = nullptr;
  bool own_stream = false;                // created here (a NULL stream cannot be captured)
  std::map<std::pair<int, unsigned>, hipGraphExec_t> graphs;  // (Krylov column, problem mask)
  int graph_pc = -1;
};

static void batch_drop_graphs(kf_batch *b) {
  for (auto &kv : b->graphs) hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

extern "C" kf_status kf_batch_create(kf_problem *const *problems, int32_t n, void *hip_stream, kf_batch **out) {
  if (!out) return fail(KF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!problems || n < 1 || n > KF_BATCH_MAX) return fail(KF_EINVAL, "batch needs 1..8 problems");
  for (int q = 0; q < n; ++q)
    if (!problems[q]) return fail(KF_EINVAL, "NULL problem in batch");
  kf_batch *b = new kf_batch();
  b->p.assign(problems, problems + n);
  b->stream = (hipStream_t)hip_stream;
  if (!b->stream) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(KF_EHIP, "hipStreamCreateWithFlags failed");
    }
    b->own_stream = true;
  }
  for (kf_problem *p : b->p) {          // the batch orders all work on one stream
    b->prev_stream.push_back(p->stream);
    p->stream = b->stream;
  }
  *out = b;
  return KF_OK;
}

extern "C" kf_status kf_batch_destroy(kf_batch *b) {
  if (!b) return KF_OK;
  hipStreamSynchronize(b->stream);
  batch_drop_graphs(b);
  for (size_t q = 0; q < b->p.size(); ++q) b->p[q]->stream = b->prev_stream[q];
  if (b->own_stream) hipStreamDestroy(b->stream);
  delete b;
  return KF_OK;
}

extern "C" kf_status kf_batch_factor(kf_batch *b, int32_t which, double *t_ms) {
  if (!b) return fail(KF_EINVAL, "batch is NULL");
  HIP_TRY(hipStreamSynchronize(b->stream));
  auto t0 = std::chrono::steady_clock::now();
  CHECK_ST(blu_factor_batch(b->p, which, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (t_ms) *t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return KF_OK;
}

extern "C" kf_status helmholtz_solve_batched(kf_batch *b, int32_t adjoint, int32_t prec, const void *const *rhs,
                                             void *const *x) {
  if (!b || !rhs || !x) return fail(KF_EINVAL, "null argument");
  for (size_t q = 0; q < b->p.size(); ++q)
    if (!rhs[q] || !x[q]) return fail(KF_EINVAL, "null field pointer");
  if (prec == KF_C128) {
    CHECK_ST(blu_factor_batch(b->p, 1, b->stream));
    CHECK_ST((blu_solve_batch<double, double2>(b->p, adjoint, (const double2 *const *)rhs, (double2 *const *)x,
                                                b->stream)));
  } else if (prec == KF_C64) {
    CHECK_ST(blu_factor_batch(b->p, 3, b->stream));
    CHECK_ST((blu_solve_batch<float, float2>(b->p, adjoint, (const float2 *const *)rhs, (float2 *const *)x,
                                              b->stream)));
  } else {
    return fail(KF_EINVAL, "batched solve supports KF_C128 and KF_C64");
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  return KF_OK;
}

// the preconditioner (eq. precond / precond_approx) and KKT matvec of Krylov column j
// for the problems in `sel`: z_j = P^-1 v_j, v_{j+1} = M z_j.  Both block solves of the
// preconditioner are single persistent launches over all selected problems.
static kf_status batch_column(kf_batch *b, const std::vector<kf_problem *> &sel, int pc, int j) {
  const size_t n = sel.size();
  std::vector<const double2 *> yu(n);
  std::vector<double2 *> zl(n), zu(n);
  for (size_t q = 0; q < n; ++q) {
    kf_problem *p = sel[q];
    const size_t N = p->Nxi, Ku = (size_t)p->K * p->Nu;
    yu[q] = p->V + (size_t)j * N;
    zu[q] = p->Z + (size_t)j * N;
    zl[q] = zu[q] + Ku + p->Ng;
  }
  if (pc == KF_PC_EXACT) CHECK_ST((blu_solve_batch<double, double2>(sel, 1, yu.data(), zl.data(), b->stream)));
  else CHECK_ST((blu_solve_batch<float, double2>(sel, 1, yu.data(), zl.data(), b->stream)));
  for (size_t q = 0; q < n; ++q) CHECK_ST(launch_precond_stage2(sel[q], sel[q]->V + (size_t)j * sel[q]->Nxi, zu[q]));
  std::vector<const double2 *> zin(zu.begin(), zu.end());
  if (pc == KF_PC_EXACT) CHECK_ST((blu_solve_batch<double, double2>(sel, 0, zin.data(), zu.data(), b->stream)));
  else CHECK_ST((blu_solve_batch<float, double2>(sel, 0, zin.data(), zu.data(), b->stream)));
  for (size_t q = 0; q < n; ++q) CHECK_ST(launch_kkt_apply(sel[q], zu[q], sel[q]->V + (size_t)(j + 1) * sel[q]->Nxi));
  return KF_OK;
}

// replay (capturing on first use) the graph of column j for the problem mask
static kf_status batch_column_graph(kf_batch *b, const std::vector<kf_problem *> &sel, unsigned mask, int pc, int j) {
  if (b->graph_pc != pc) { batch_drop_graphs(b); b->graph_pc = pc; }
  auto key = std::make_pair(j, mask);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    std::vector<bool> prof(sel.size());
    for (size_t q = 0; q < sel.size(); ++q) { prof[q] = sel[q]->prof; sel[q]->prof = false; }
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    kf_status st = batch_column(b, sel, pc, j);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    for (size_t q = 0; q < sel.size(); ++q) sel[q]->prof = prof[q];
    if (st != KF_OK) { if (graph) hipGraphDestroy(graph); return st; }
    if (e != hipSuccess) return fail(KF_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(KF_EHIP, std::string("graph instantiate failed: ") + hipGetErrorString(e));
    it = b->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, b->stream));
  return KF_OK;
}

// One full-space Gauss-Newton step for every problem of the batch: the factorisations,
// background solves and every preconditioner application run as persistent launches
// over all problems; the FGMRES iterations of the problems advance in lockstep, the
// preconditioner + KKT matvec of each Krylov column replayed from a captured hipGraph
// (use_graph != 0).  Each problem keeps its own Krylov scalars and stops at its own
// tolerance.  Arrays d_obs, xi_out, gamma_next and st have one entry per problem.
extern "C" kf_status newton_step_batched(kf_batch *b, const void *const *d_obs, const kf_newton_opts *o,
                                         void *const *xi_out, double *const *gamma_next, int32_t update_in_place,
                                         int32_t use_graph, kf_newton_stats *st) {
  if (!b || !d_obs || !o) return fail(KF_EINVAL, "null argument");
  const int n = (int)b->p.size();
  for (int q = 0; q < n; ++q) if (!d_obs[q]) return fail(KF_EINVAL, "null d_obs entry");
  if (!(o->rtol > 0.0) || o->restart < 1 || o->restart > 200 || o->maxit < 1)
    return fail(KF_EINVAL, "need rtol > 0, 1 <= restart <= 200, maxit >= 1");
  if (o->pc != KF_PC_EXACT && o->pc != KF_PC_INEXACT) return fail(KF_EINVAL, "invalid preconditioner");
  if (o->fwd_prec != KF_C128) return fail(KF_EINVAL, "batched steps use a complex128 background solve");
  if (o->outer != KF_OUTER_FGMRES) return fail(KF_EINVAL, "batched steps use flexible GMRES");
  if (!(o->reorth_eta >= 0.0 && o->reorth_eta <= 1.0)) return fail(KF_EINVAL, "reorth_eta must be in [0, 1]");
  const int m = o->restart;
  auto T0 = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  std::vector<kf_newton_stats> S(n);
  for (auto &s : S) { std::memset(&s, 0, sizeof(s)); s.misfit_after = -1.0; }
  for (kf_problem *p : b->p) CHECK_ST(ensure_krylov(p, m));
  HIP_TRY(hipStreamSynchronize(b->stream));
  auto t = std::chrono::steady_clock::now();
  CHECK_ST(blu_factor_batch(b->p, o->pc == KF_PC_INEXACT ? 3 : 1, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  const double t_fac = ms_since(t);
  t = std::chrono::steady_clock::now();
  {
    std::vector<const double2 *> f(n);
    std::vector<double2 *> u(n);
    for (int q = 0; q < n; ++q) {
      CHECK_ST(launch_sources(b->p[q], b->p[q]->vec_c));
      f[q] = b->p[q]->vec_c;
      u[q] = b->p[q]->u_n;
    }
    CHECK_ST((blu_solve_batch<double, double2>(b->p, 0, f.data(), u.data(), b->stream)));
    for (kf_problem *p : b->p) p->have_un = true;
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  const double t_fwd = ms_since(t);
  // residuals and right-hand sides
  std::vector<double> bnorm(n), dn(n);
  kf_status e = KF_OK;
  for (int q = 0; q < n; ++q) {
    kf_problem *p = b->p[q];
    CHECK_ST(launch_residual(p, (const double2 *)d_obs[q], p->u_n, p->d_r, p->d_wr));
    const int64_t nd = (int64_t)p->K * p->nrec;
    double rn = host_norm(p, p->d_r, nd, &e); CHECK_ST(e);
    dn[q] = host_norm(p, (const double2 *)d_obs[q], nd, &e); CHECK_ST(e);
    double wn = host_norm(p, p->d_wr, nd, &e); CHECK_ST(e);
    S[q].misfit_before = dn[q] > 0 ? rn / dn[q] : rn;
    S[q].phi_before = 0.5 * wn * wn;
    CHECK_ST(launch_rhs(p, p->d_r, p->d_rptr, p->d_rlist, p->xi_b, p->d.reg_on_update));
    bnorm[q] = host_norm(p, p->xi_b, p->Nxi, &e); CHECK_ST(e);
    HIP_TRY(hipMemsetAsync(p->xi_x, 0, sizeof(double2) * p->Nxi, b->stream));
    S[q].t_factor_ms = t_fac;
    S[q].t_forward_ms = t_fwd;
  }
  // lockstep flexible GMRES
  std::vector<bool> done(n, false);
  std::vector<int> total(n, 0), reorth(n, 0);
  std::vector<std::vector<double>> hist(n);
  kf_status status = KF_OK;
  for (int q = 0; q < n; ++q) if (bnorm[q] == 0.0) { done[q] = true; S[q].rel_res = 0.0; }
  double t_cols = 0.0, t_orth = 0.0;
  for (;;) {
    // true residual at the start of each cycle
    std::vector<int> act;
    for (int q = 0; q < n; ++q) {
      if (done[q]) continue;
      kf_problem *p = b->p[q];
      const int64_t N = p->Nxi;
      double2 *H = p->hess;
      double2 *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *h1 = g + (m + 1), *h2 = h1 + (m + 1),
              *y = h2 + (m + 1);
      double *scal = (double *)(y + m + 8);
      (void)cs; (void)sn; (void)h1; (void)h2;
      HIP_TRY(hipMemcpyAsync(p->V, p->xi_b, sizeof(double2) * N, hipMemcpyDeviceToDevice, b->stream));
      if (total[q] > 0) {
        CHECK_ST(launch_kkt_apply(p, p->xi_x, p->xi_w));
        CHECK_ST(launch_axpy_field(p, N, make_double2(-1.0, 0.0), p->xi_w, p->V));
      }
      CHECK_ST(norm_c128(p, p->V, N, scal + 1));
      HIP_TRY(hipMemcpyAsync(p->host_pinned, scal + 1, sizeof(double), hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
      const double beta = p->host_pinned[0];
      if (!std::isfinite(beta)) { status = fail(KF_ENAN, "non-finite residual in batched FGMRES"); done[q] = true; continue; }
      S[q].rel_res = beta / bnorm[q];
      if (S[q].rel_res <= o->rtol) { done[q] = true; continue; }
      if (total[q] >= o->maxit) { status = fail(KF_ENOCONV, "batched FGMRES reached maxit"); done[q] = true; continue; }
      CHECK_ST(scale_inv(p, N, scal + 1, p->V, p->V));
      CHECK_ST(set_g0(p, m, scal + 1, g));
      act.push_back(q);
    }
    if (act.empty()) break;
    std::vector<int> nj(n, 0);
    std::vector<bool> live(n, false);
    for (int q : act) live[q] = true;
    for (int j = 0; j < m; ++j) {
      std::vector<kf_problem *> sel;
      unsigned mask = 0;
      for (int q : act) { sel.push_back(b->p[q]); mask |= 1u << q; }
      auto tc = std::chrono::steady_clock::now();
      if (use_graph) CHECK_ST(batch_column_graph(b, sel, mask, o->pc, j));
      else CHECK_ST(batch_column(b, sel, o->pc, j));
      HIP_TRY(hipStreamSynchronize(b->stream));
      t_cols += ms_since(tc);
      tc = std::chrono::steady_clock::now();
      for (int q : act) {
        kf_problem *p = b->p[q];
        if (!live[q]) continue;
        const int64_t N = p->Nxi;
        double2 *H = p->hess;
        double2 *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *h1 = g + (m + 1), *h2 = h1 + (m + 1),
                *y = h2 + (m + 1);
        double *scal = (double *)(y + m + 8);
        double2 *Vn = p->V + (size_t)(j + 1) * N;
        CHECK_ST(gram_schmidt(p, j, Vn, h1, h2, scal, o->reorth_eta));
        CHECK_ST(arnoldi_finish(p, j, m, h1, h2, scal + 0, H, cs, sn, g, scal + 2));
        HIP_TRY(hipMemcpyAsync(p->host_pinned, scal, 7 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        const double hn = p->host_pinned[0], est = p->host_pinned[2] / bnorm[q];
        reorth[q] += *(const int *)(p->host_pinned + 6);
        total[q] += 1;
        nj[q] = j + 1;
        hist[q].push_back(est);
        if (!std::isfinite(est) || !std::isfinite(hn)) { status = fail(KF_ENAN, "non-finite value in Arnoldi"); live[q] = false; }
        else if (hn == 0.0 || est <= o->rtol || total[q] >= o->maxit) live[q] = false;
      }
      t_orth += ms_since(tc);
      bool any = false;
      for (int q : act) any = any || live[q];
      if (!any) break;
    }
    for (int q : act) {
      kf_problem *p = b->p[q];
      double2 *H = p->hess;
      double2 *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *h1 = g + (m + 1), *h2 = h1 + (m + 1),
              *y = h2 + (m + 1);
      (void)cs; (void)sn; (void)h1; (void)h2;
      CHECK_ST(hess_backsolve(p, nj[q], m, H, g, y));
      CHECK_ST(multiaxpy_c128(p, p->Z, nj[q], y, 1.0, p->xi_x, p->Nxi));
      S[q].restarts += 1;
    }
  }
  // updates and statistics
  for (int q = 0; q < n; ++q) {
    kf_problem *p = b->p[q];
    const size_t Ku = (size_t)p->K * p->Nu;
    const double2 *ds = p->xi_x + Ku;
    S[q].outer_iters = total[q];
    S[q].reorth_passes = reorth[q];
    for (size_t r = 0; r < hist[q].size() && r < 512; ++r) S[q].rel_res_hist[r] = hist[q][r];
    double dsn = host_norm(p, ds, p->Ng, &e); CHECK_ST(e);
    CHECK_ST(imag_part(p, p->Ng, ds, p->vec_a));
    double dsi = host_norm(p, p->vec_a, p->Ng, &e); CHECK_ST(e);
    S[q].ds_imag_ratio = dsn > 0 ? dsi / dsn : 0.0;
    if (xi_out && xi_out[q])
      HIP_TRY(hipMemcpyAsync(xi_out[q], p->xi_x, sizeof(double2) * p->Nxi, hipMemcpyDeviceToDevice, b->stream));
    if (gamma_next && gamma_next[q]) {
      HIP_TRY(hipMemcpyAsync(gamma_next[q], p->gamma, sizeof(double) * p->Nu, hipMemcpyDeviceToDevice, b->stream));
      CHECK_ST(launch_update_gamma(p, ds, gamma_next[q]));
    }
    if (update_in_place) {
      CHECK_ST(launch_update_gamma(p, ds, p->gamma));
      p->have_T64 = p->have_T32 = false;
      ++p->gamma_version;
    }
    S[q].t_precond_ms = t_cols;    // columns (preconditioner + matvec) of all problems together
    S[q].t_orth_ms = t_orth;
  }
  if (update_in_place) batch_drop_graphs(b);   // the captured solves refer to factors about to change
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int q = 0; q < n; ++q) {
    S[q].t_total_ms = ms_since(T0);
    if (st) st[q] = S[q];
  }
  return status;
}
