// C ABI of libcsc: argument validation, graph handles, host FP64 math (Chebyshev
// coefficients, eigencount dichotomy), timing, and the entry points that enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "csc_internal.h"

namespace csc {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

csc_status fail(csc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// ------------------------------------------------------------------------------------
// Chebyshev coefficients of the step 1[lambda <= lambda_c] on [0, lmax] (Sec. 3.2):
// with x = cos(theta), the step is 1[theta >= theta_c]; its Chebyshev series has
// c_j = (2 / pi) int_{theta_c}^{pi} cos(j theta) d theta, folded so that a_0 = c_0 / 2.
// Jackson damping factor for m + 1 terms (Weisse et al., Rev. Mod. Phys. 78, 2006):
// g_j = ((M - j) cos(pi j / M) + sin(pi j / M) cot(pi / M)) / M with M = m + 2.
void cheb_coeffs(int m, double lmax, double lambda_c, csc_damping damp, double* a) {
  double x = 2.0 * lambda_c / lmax - 1.0;
  x = std::min(1.0, std::max(-1.0, x));
  const double th = std::acos(x);
  a[0] = 1.0 - th / M_PI;
  for (int j = 1; j <= m; ++j) a[j] = -2.0 * std::sin(j * th) / (j * M_PI);
  if (damp == CSC_DAMP_JACKSON) {
    const double M = m + 2.0;
    const double cot = std::cos(M_PI / M) / std::sin(M_PI / M);
    for (int j = 0; j <= m; ++j)
      a[j] *= ((M - j) * std::cos(M_PI * j / M) + std::sin(M_PI * j / M) * cot) / M;
  }
}

// Fixed-step dichotomy on the Hutchinson count c(lambda) = sum_j a_j(lambda) mu_j /
// (sigma2 n_probe): lo moves up when c(mid) < k, hi moves down otherwise; returns hi.
void bisect_moments(const double* mu, int m, double lmax, csc_damping damp, double sigma2,
                    int n_probe, double k, int n_cand, double lo, double hi, double* lambda_c,
                    double* count, double* trace) {
  std::vector<double> a(m + 1);
  auto c = [&](double lam) {
    cheb_coeffs(m, lmax, lam, damp, a.data());
    double s = 0.0;
    for (int j = 0; j <= m; ++j) s += a[j] * mu[j];
    return s / (sigma2 * n_probe);
  };
  for (int i = 0; i < n_cand; ++i) {
    const double mid = 0.5 * (lo + hi);
    const double cm = c(mid);
    if (trace) {
      trace[2 * i] = mid;
      trace[2 * i + 1] = cm;
    }
    if (cm < k) lo = mid;
    else hi = mid;
  }
  *lambda_c = hi;
  if (count) *count = c(hi);
}

// ------------------------------------------------------------------------------------
// timing: pairs of events around the recurrence-step launches

namespace {
struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;
  std::vector<hipEvent_t> pool;
  hipEvent_t pending = nullptr;
  int64_t launches = 0;
  double bytes = 0.0;
};
Timing g_timing;

hipEvent_t take_event() {
  if (!g_timing.pool.empty()) {
    hipEvent_t e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

void timing_begin(hipStream_t s) {
  if (!g_timing.on) return;
  g_timing.pending = take_event();
  if (g_timing.pending) hipEventRecord(g_timing.pending, s);
}

void timing_end(hipStream_t s, int64_t launches, double bytes) {
  if (!g_timing.on || !g_timing.pending) return;
  hipEvent_t e = take_event();
  if (!e) return;
  hipEventRecord(e, s);
  g_timing.pairs.emplace_back(g_timing.pending, e);
  g_timing.pending = nullptr;
  g_timing.launches += launches;
  g_timing.bytes += bytes;
}

// ------------------------------------------------------------------------------------
// dynamic state and adjoint live in their own translation units
csc_status dyn_create(int64_t n, int d, int k, double p, int m, csc_damping damp,
                      csc_dtype feat_dt, uint64_t seed, const csc_dyn_opts* opts, csc_dyn* out);
csc_status dyn_step(csc_dyn st, csc_graph g, int32_t* labels, double* lambda_t, int* refined,
                    double* count, void* stream);
csc_status dyn_steps(csc_dyn st, const csc_graph* graphs, int S, int32_t* const* labels,
                     double* lambdas, int* refined, double* counts, void* stream);
csc_status dyn_features(csc_dyn st, const void** theta, csc_dtype* dt, int64_t* ld,
                        const float** centroids);
csc_status dyn_similarity(csc_dyn st, int t, double* rho_edge, double* rho_hat, int* refreshed);
size_t dyn_state_bytes(csc_dyn st);
csc_status dyn_export(csc_dyn st, void* buf, size_t bytes, hipStream_t s);
csc_status dyn_import(csc_dyn st, const void* buf, size_t bytes, hipStream_t s);
csc_status dyn_destroy(csc_dyn st);
size_t backward_workspace(int64_t n, int w, int m, int ckpt);
csc_status run_backward(const Graph* g, double lmax, int m, const double* a, const float* X,
                        int64_t ldx, const float* G, int64_t ldg, int w, float* dX, int64_t lddx,
                        double* da, float* dA, int ckpt, void* work, size_t work_bytes,
                        hipStream_t s);

}  // namespace csc

using namespace csc;

extern "C" {

const char* csc_last_error(void) { return g_err.c_str(); }

int csc_version(void) { return 10000; }

// ------------------------------------------------------------------------------------
// graph

csc_status csc_graph_create(int64_t n, int64_t nnz, int64_t nnz_capacity,
                            const int64_t* rowptr_d, const int32_t* colidx_d, const double* w_d,
                            csc_dtype val_dt, csc_laplacian lap, int validate, void* stream,
                            csc_graph* out) {
  if (!out) return fail(CSC_E_ARG, "out is null");
  *out = nullptr;
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(CSC_E_ARG, "n must be in [1, 2^31)");
  if (nnz < 0 || nnz_capacity < nnz || nnz_capacity >= (int64_t(1) << 31))
    return fail(CSC_E_ARG, "need 0 <= nnz <= nnz_capacity < 2^31");
  if (!rowptr_d || (nnz > 0 && (!colidx_d || !w_d))) return fail(CSC_E_ARG, "null CSR array");
  if (val_dt != CSC_F32 && val_dt != CSC_BF16) return fail(CSC_E_DTYPE, "values must be F32 or BF16");
  if (lap != CSC_LAP_NORMALIZED && lap != CSC_LAP_COMBINATORIAL)
    return fail(CSC_E_ARG, "unknown Laplacian kind");
  auto* h = new csc_graph_s();
  Graph& g = h->g;
  g.n = n;
  g.cap = std::max<int64_t>(nnz_capacity, 1);
  g.val_dt = val_dt;
  g.lap = lap;
  const bool comb = lap == CSC_LAP_COMBINATORIAL;
  bool ok = hipMalloc(&g.rowptr, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            hipMalloc(&g.colidx, sizeof(int32_t) * g.cap) == hipSuccess &&
            hipMalloc(&g.vals, dtype_size(val_dt) * g.cap) == hipSuccess &&
            hipMalloc(&g.dinv, sizeof(double) * n) == hipSuccess &&
            hipMalloc(&g.mirror, sizeof(int32_t) * g.cap) == hipSuccess &&
            hipMalloc(&g.flags, sizeof(int32_t) * 4) == hipSuccess &&
            (!comb || (hipMalloc(&g.diag, sizeof(float) * n) == hipSuccess &&
                       hipMalloc(&g.deg, sizeof(double) * n) == hipSuccess));
  if (!ok) {
    csc_graph_destroy(h);
    return fail(CSC_E_NOMEM, "device allocation failed in csc_graph_create");
  }
  csc_status st = graph_build(&g, nnz, rowptr_d, colidx_d, w_d, validate, as_stream(stream));
  if (st != CSC_OK) {
    std::string msg = g_err;
    csc_graph_destroy(h);
    return fail(st, msg);
  }
  *out = h;
  return CSC_OK;
}

csc_status csc_graph_update(csc_graph h, int64_t nnz, const int64_t* rowptr_d,
                            const int32_t* colidx_d, const double* w_d, int validate,
                            void* stream) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (nnz < 0 || nnz > h->g.cap) return fail(CSC_E_ARG, "nnz exceeds the handle's capacity");
  if (!rowptr_d || (nnz > 0 && (!colidx_d || !w_d))) return fail(CSC_E_ARG, "null CSR array");
  return graph_build(&h->g, nnz, rowptr_d, colidx_d, w_d, validate, as_stream(stream));
}

csc_status csc_graph_destroy(csc_graph h) {
  if (!h) return CSC_OK;
  Graph& g = h->g;
  if (g.rowptr) (void)hipFree(g.rowptr);
  if (g.colidx) (void)hipFree(g.colidx);
  if (g.vals) (void)hipFree(g.vals);
  if (g.dinv) (void)hipFree(g.dinv);
  if (g.mirror) (void)hipFree(g.mirror);
  if (g.flags) (void)hipFree(g.flags);
  if (g.diag) (void)hipFree(g.diag);
  if (g.deg) (void)hipFree(g.deg);
  delete h;
  return CSC_OK;
}

csc_status csc_graph_info(csc_graph h, int64_t* n, int64_t* nnz, int64_t* isolated) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (n) *n = h->g.n;
  if (nnz) *nnz = h->g.nnz;
  if (isolated) {
    int32_t v = 0;
    CSC_HIP(hipDeviceSynchronize());
    CSC_HIP(hipMemcpy(&v, h->g.flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
    *isolated = v;
  }
  return CSC_OK;
}

csc_status csc_graph_arrays(csc_graph h, const int32_t** rowptr, const int32_t** colidx,
                            void** vals, csc_dtype* val_dt, const double** dinv,
                            const int32_t** mirror) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (mirror) {
    CSC_TRY(graph_ensure_mirror(&h->g, nullptr));
    CSC_HIP(hipStreamSynchronize(nullptr));
  }
  if (rowptr) *rowptr = h->g.rowptr;
  if (colidx) *colidx = h->g.colidx;
  if (vals) *vals = h->g.vals;
  if (val_dt) *val_dt = h->g.val_dt;
  if (dinv) *dinv = h->g.dinv;
  if (mirror) *mirror = h->g.mirror;
  return CSC_OK;
}

size_t csc_weight_grad_workspace_bytes(int64_t n) { return align_up(static_cast<size_t>(std::max<int64_t>(n, 1)) * 8); }

csc_status csc_weight_grad(csc_graph g, const float* dA, double* dW, void* work, size_t work_bytes,
                           void* stream) {
  if (!g || !dA || !dW) return fail(CSC_E_ARG, "null argument");
  if (!work || work_bytes < csc_weight_grad_workspace_bytes(g->g.n)) return fail(CSC_E_ARG, "workspace too small");
  return graph_weight_grad(&g->g, dA, dW, static_cast<double*>(work), as_stream(stream));
}

csc_status csc_graph_distance(csc_graph g1, csc_graph g2, double* rho, void* stream) {
  if (!g1 || !g2 || !rho) return fail(CSC_E_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  const size_t wb = distance_workspace(g1->g.n) + 256;
  void* buf = nullptr;
  if (hipMalloc(&buf, wb) != hipSuccess) return fail(CSC_E_NOMEM, "csc_graph_distance: allocation failed");
  double* out = static_cast<double*>(buf);
  csc_status st = graph_distance2(&g1->g, &g2->g, out, static_cast<char*>(buf) + 256, wb - 256, s);
  double v = 0.0;
  if (st == CSC_OK && (hipMemcpyAsync(&v, out, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                       hipStreamSynchronize(s) != hipSuccess))
    st = fail(CSC_E_HIP, "csc_graph_distance: copy failed");
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (st == CSC_OK) *rho = std::sqrt(v);
  return st;
}

size_t csc_compressive_workspace_bytes(int64_t n, int d, int k, int n_sample) {
  if (n < 1 || d < 1 || k < 1 || n_sample < 1) return 0;
  return compressive_workspace(n, d, k, n_sample);
}

csc_status csc_compressive_kmeans(csc_graph g, const void* F, csc_dtype f_dt, int64_t ldf, int d,
                                  int k, int n_sample, int r, double gamma, int lloyd_iters,
                                  int cg_iters, double cg_tol, uint64_t seed,
                                  uint64_t sample_stream, uint64_t kmeans_stream, int32_t* labels,
                                  int32_t* samples, int32_t* sample_labels, float* X,
                                  int* cg_iters_done, void* work, size_t work_bytes, void* stream) {
  if (!g) return fail(CSC_E_ARG, "null graph");
  if (lloyd_iters < 0 || lloyd_iters > 1024) return fail(CSC_E_ARG, "lloyd_iters must be in [0, 1024]");
  return run_compressive(&g->g, F, f_dt, ldf, d, k, n_sample, r, gamma, lloyd_iters, cg_iters,
                         cg_tol, seed, sample_stream, kmeans_stream, labels, samples,
                         sample_labels, X, cg_iters_done, work, work_bytes, as_stream(stream));
}

csc_status csc_lmax(csc_graph h, int iters, double* lmax, void* stream) {
  if (!h || !lmax) return fail(CSC_E_ARG, "null argument");
  if (iters < 0) return fail(CSC_E_ARG, "iters must be >= 0");
  const Graph& g = h->g;
  if (iters == 0) {
    *lmax = g.lmax_bound;
    return CSC_OK;
  }
  hipStream_t s = as_stream(stream);
  // Power iteration on L.  One application of L is the degree-1 filter
  // a0 T_0 + a1 T_1(L~) with lmax = 2 (L~ = L - I) and a0 = a1 = 1.
  const size_t fw = filter_workspace(g.n, 1, CSC_F32);
  const size_t dw = dot_workspace(g.n);
  void* buf = nullptr;
  if (hipMalloc(&buf, 2 * align_up(g.n * sizeof(double)) + fw + dw + 512) != hipSuccess)
    return fail(CSC_E_NOMEM, "csc_lmax: allocation failed");
  char* base = static_cast<char*>(buf);
  double* x = reinterpret_cast<double*>(base);
  double* y = reinterpret_cast<double*>(base + align_up(g.n * sizeof(double)));
  void* fwork = base + 2 * align_up(g.n * sizeof(double));
  void* dwork = static_cast<char*>(fwork) + fw;
  double* res = reinterpret_cast<double*>(static_cast<char*>(dwork) + dw);
  csc_status st = launch_randn(x, CSC_F64, g.n, 1, 1, 0, 0x5eedull, 0x1a3aull, 1.0, s);
  double rq = 0.0, resid = 0.0;
  for (int it = 0; st == CSC_OK && it < iters; ++it) {
    double nrm2 = 0.0;
    st = launch_dot(x, CSC_F64, 1, x, CSC_F64, 1, g.n, 1, res, dwork, dw, s);
    if (st != CSC_OK) break;
    if (hipMemcpyAsync(&nrm2, res, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(CSC_E_HIP, "csc_lmax: copy failed");
      break;
    }
    const double inv = 1.0 / std::sqrt(std::max(nrm2, 1e-300));
    const double a[2] = {inv, inv};
    st = run_filter(&g, 2.0, 1, a, x, CSC_F64, 1, y, CSC_F64, 1, 1, CSC_F32, nullptr, 0, fwork,
                    fw, s);
    if (st != CSC_OK) break;
    // Rayleigh quotient rho of the normalised x and the residual |L x^ - rho x^|, from
    // <x, y> / |x| and <y, y> with y = L x / |x|
    double xy = 0.0, yy = 0.0;
    st = launch_dot(x, CSC_F64, 1, y, CSC_F64, 1, g.n, 1, res, dwork, dw, s);
    if (st == CSC_OK) st = launch_dot(y, CSC_F64, 1, y, CSC_F64, 1, g.n, 1, res + 1, dwork, dw, s);
    if (st != CSC_OK) break;
    double two[2];
    if (hipMemcpyAsync(two, res, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(CSC_E_HIP, "csc_lmax: copy failed");
      break;
    }
    xy = two[0];
    yy = two[1];
    rq = xy * inv;
    resid = std::sqrt(std::max(0.0, yy - rq * rq));
    std::swap(x, y);
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (st != CSC_OK) return st;
  *lmax = std::min(g.lmax_bound, 1.01 * (rq + resid));
  return CSC_OK;
}

// ------------------------------------------------------------------------------------
// coefficients, filter, moments, eigencount

csc_status csc_cheb_coeffs(int m, double lmax, double lambda_c, csc_damping damp, double* a) {
  if (m < 0 || !a) return fail(CSC_E_ARG, "need m >= 0 and a non-null output");
  if (!(lmax > 0.0)) return fail(CSC_E_ARG, "lmax must be > 0");
  if (!(lambda_c >= 0.0 && lambda_c <= lmax)) return fail(CSC_E_ARG, "lambda_c must be in [0, lmax]");
  if (damp != CSC_DAMP_NONE && damp != CSC_DAMP_JACKSON) return fail(CSC_E_ARG, "bad damping");
  cheb_coeffs(m, lmax, lambda_c, damp, a);
  return CSC_OK;
}

size_t csc_cheb_filter_workspace_bytes(int64_t n, int w, csc_dtype iter_dt) {
  return filter_workspace(n, w, iter_dt);
}

csc_status csc_cheb_filter(csc_graph h, double lmax, int m, const double* a, const void* X,
                           csc_dtype x_dt, int64_t ldx, void* Y, csc_dtype y_dt, int64_t ldy,
                           int w, csc_dtype iter_dt, double* moments, void* work,
                           size_t work_bytes, void* stream) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (!a) return fail(CSC_E_ARG, "null coefficients");
  if (m > 4096) return fail(CSC_E_ARG, "m must be <= 4096");
  return run_filter(&h->g, lmax, m, a, X, x_dt, ldx, Y, y_dt, ldy, w, iter_dt, moments, 0, work,
                    work_bytes, as_stream(stream));
}

csc_status csc_cheb_moments(csc_graph h, double lmax, int m, const void* P, csc_dtype p_dt,
                            int64_t ldp, int n_probe, csc_dtype iter_dt, double* moments,
                            void* work, size_t work_bytes, void* stream) {
  if (!h || !moments) return fail(CSC_E_ARG, "null argument");
  if (m < 1 || m > 4096) return fail(CSC_E_ARG, "m must be in [1, 4096]");
  return run_filter(&h->g, lmax, m, nullptr, P, p_dt, ldp, nullptr, CSC_F32, 0, n_probe, iter_dt,
                    moments, 1, work, work_bytes, as_stream(stream));
}

csc_status csc_eigcount_from_moments(const double* mu, int m, double lmax, csc_damping damp,
                                     double sigma2, int n_probe, double k, int n_cand, double lo,
                                     double hi, double* lambda_c, double* count, double* trace) {
  if (!mu || !lambda_c) return fail(CSC_E_ARG, "null argument");
  if (m < 1 || n_cand < 0 || n_probe < 1 || !(sigma2 > 0.0) || !(lmax > 0.0))
    return fail(CSC_E_ARG, "bad eigencount parameters");
  if (!(lo >= 0.0 && lo <= hi && hi <= lmax)) return fail(CSC_E_ARG, "need 0 <= lo <= hi <= lmax");
  bisect_moments(mu, m, lmax, damp, sigma2, n_probe, k, n_cand, lo, hi, lambda_c, count, trace);
  return CSC_OK;
}

csc_status csc_eigcount(csc_graph h, double lmax, int m, csc_damping damp, const void* P,
                        csc_dtype p_dt, int64_t ldp, int n_probe, double sigma2, double k,
                        int n_cand, double lo, double hi, csc_dtype iter_dt, double* lambda_c,
                        double* count, double* trace, double* moments_out, void* work,
                        size_t work_bytes, void* stream) {
  if (!h || !lambda_c) return fail(CSC_E_ARG, "null argument");
  if (m < 1 || m > 4096) return fail(CSC_E_ARG, "m must be in [1, 4096]");
  if (!(lo >= 0.0 && lo <= hi && hi <= lmax)) return fail(CSC_E_ARG, "need 0 <= lo <= hi <= lmax");
  hipStream_t s = as_stream(stream);
  // moments go to the tail of the workspace
  const size_t need = filter_workspace(h->g.n, n_probe, iter_dt);
  const size_t mom_bytes = align_up(sizeof(double) * (m + 1));
  if (!work || work_bytes < need + mom_bytes)
    return fail(CSC_E_ARG, "workspace too small: need " + std::to_string(need + mom_bytes));
  double* mu_d = reinterpret_cast<double*>(static_cast<char*>(work) + need);
  CSC_TRY(run_filter(&h->g, lmax, m, nullptr, P, p_dt, ldp, nullptr, CSC_F32, 0, n_probe,
                     iter_dt, mu_d, 1, work, need, s));
  std::vector<double> mu(m + 1);
  CSC_HIP(hipMemcpyAsync(mu.data(), mu_d, sizeof(double) * (m + 1), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  if (moments_out) std::memcpy(moments_out, mu.data(), sizeof(double) * (m + 1));
  return csc_eigcount_from_moments(mu.data(), m, lmax, damp, sigma2, n_probe, k, n_cand, lo, hi,
                                   lambda_c, count, trace);
}

size_t csc_dot_workspace_bytes(int64_t n) { return dot_workspace(n); }

csc_status csc_dot(const void* X, csc_dtype x_dt, int64_t ldx, const void* Y, csc_dtype y_dt,
                   int64_t ldy, int64_t n, int w, double* result, void* work, size_t work_bytes,
                   void* stream) {
  if (!X || !Y || !result) return fail(CSC_E_ARG, "null argument");
  return launch_dot(X, x_dt, ldx, Y, y_dt, ldy, n, w, result, work, work_bytes, as_stream(stream));
}

csc_status csc_randn(void* X, csc_dtype dt, int64_t n, int w, int64_t ldx, int64_t row0,
                     uint64_t seed, uint64_t stream_id, double sigma, void* stream) {
  return launch_randn(X, dt, n, w, ldx, row0, seed, stream_id, sigma, as_stream(stream));
}

csc_status csc_uniforms(double* u, int count, uint64_t seed, uint64_t stream_id, void* stream) {
  return launch_uniforms(u, count, seed, stream_id, as_stream(stream));
}

// ------------------------------------------------------------------------------------
// k-means

size_t csc_kmeans_workspace_bytes(int64_t n, int d, int k) { return kmeans_workspace(n, d, k); }

csc_status csc_kmeans_assign(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                             const float* C, int k, int32_t* labels, float* best_d2,
                             float* sums, int32_t* counts, void* work, size_t work_bytes,
                             void* stream) {
  return launch_kmeans_assign(F, f_dt, ldf, n, d, C, k, labels, best_d2, sums, counts, work,
                              work_bytes, as_stream(stream));
}

csc_status csc_kmeans_assign_noalloc(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n,
                                     int d, const float* C, int k, int32_t* labels,
                                     float* best_d2, void* stream) {
  return launch_kmeans_assign_static(F, f_dt, ldf, n, d, C, k, labels, best_d2,
                                     as_stream(stream));
}

csc_status csc_kmeans_update(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                             const int32_t* labels, int k, float* C, int32_t* counts, void* work,
                             size_t work_bytes, void* stream) {
  if (!labels || !C) return fail(CSC_E_ARG, "null argument");
  return launch_kmeans_update(F, f_dt, ldf, n, d, labels, k, C, counts, work, work_bytes,
                              as_stream(stream));
}

csc_status csc_kmeans_seed(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                           const double* u, float* C, int32_t* idx, void* work,
                           size_t work_bytes, void* stream) {
  if (!u || !C) return fail(CSC_E_ARG, "null argument");
  return launch_kmeans_seed(F, f_dt, ldf, n, d, k, u, C, idx, work, work_bytes,
                            as_stream(stream));
}

csc_status csc_kmeans(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                      int iters, int init, uint64_t seed, uint64_t stream_id, float* C,
                      int32_t* labels, double* objective, void* work, size_t work_bytes,
                      void* stream) {
  if (!C || !labels) return fail(CSC_E_ARG, "null argument");
  if (init != 0 && init != 1) return fail(CSC_E_ARG, "init must be 0 (k-means++) or 1 (given)");
  return run_kmeans(F, f_dt, ldf, n, d, k, iters, init, seed, stream_id, C, labels, objective,
                    work, work_bytes, as_stream(stream));
}

// ------------------------------------------------------------------------------------
// dynamic CSC

csc_status csc_dyn_create(int64_t n, int d, int k, double p, int m, csc_damping damp,
                          csc_dtype feat_dt, uint64_t seed, const csc_dyn_opts* opts,
                          csc_dyn* out) {
  return dyn_create(n, d, k, p, m, damp, feat_dt, seed, opts, out);
}

csc_status csc_dynamic_step(csc_dyn st, csc_graph g, int32_t* labels, double* lambda_t,
                            int* refined, double* count, void* stream) {
  return dyn_step(st, g, labels, lambda_t, refined, count, stream);
}

csc_status csc_dynamic_steps(csc_dyn st, const csc_graph* graphs, int S, int32_t* const* labels,
                             double* lambdas, int* refined, double* counts, void* stream) {
  return dyn_steps(st, graphs, S, labels, lambdas, refined, counts, stream);
}

csc_status csc_dyn_features(csc_dyn st, const void** theta, csc_dtype* dt, int64_t* ld,
                            const float** centroids) {
  return dyn_features(st, theta, dt, ld, centroids);
}

csc_status csc_dyn_similarity(csc_dyn st, int t, double* rho_edge, double* rho_hat,
                              int* refreshed) {
  return dyn_similarity(st, t, rho_edge, rho_hat, refreshed);
}

size_t csc_dyn_state_bytes(csc_dyn st) { return dyn_state_bytes(st); }

csc_status csc_dyn_export(csc_dyn st, void* host_buf, size_t bytes, void* stream) {
  return dyn_export(st, host_buf, bytes, as_stream(stream));
}

csc_status csc_dyn_import(csc_dyn st, const void* host_buf, size_t bytes, void* stream) {
  return dyn_import(st, host_buf, bytes, as_stream(stream));
}

csc_status csc_dyn_destroy(csc_dyn st) { return dyn_destroy(st); }

// ------------------------------------------------------------------------------------
// adjoint

size_t csc_cheb_backward_workspace_bytes(int64_t n, int w, int m, int ckpt_every) {
  return backward_workspace(n, w, m, ckpt_every);
}

csc_status csc_cheb_filter_backward(csc_graph h, double lmax, int m, const double* a,
                                    const float* X, int64_t ldx, const float* G, int64_t ldg,
                                    int w, float* dX, int64_t lddx, double* da, float* dA,
                                    int ckpt_every, void* work, size_t work_bytes,
                                    void* stream) {
  if (!h || !a || !X || !G) return fail(CSC_E_ARG, "null argument");
  if (h->g.lap != CSC_LAP_NORMALIZED)
    return fail(CSC_E_ARG, "the adjoint is defined for the normalized Laplacian");
  CSC_TRY(graph_ensure_mirror(&h->g, as_stream(stream)));
  return run_backward(&h->g, lmax, m, a, X, ldx, G, ldg, w, dX, lddx, da, dA, ckpt_every, work,
                      work_bytes, as_stream(stream));
}

// ------------------------------------------------------------------------------------
// measurement and kernel shapes

csc_status csc_timing_enable(int on) {
  g_timing.on = on != 0;
  return CSC_OK;
}

csc_status csc_timing_reset(void) {
  for (auto& p : g_timing.pairs) {
    g_timing.pool.push_back(p.first);
    g_timing.pool.push_back(p.second);
  }
  g_timing.pairs.clear();
  g_timing.launches = 0;
  g_timing.bytes = 0.0;
  return CSC_OK;
}

csc_status csc_timing_read(double* ms, int64_t* launches, double* bytes) {
  double total = 0.0;
  for (auto& p : g_timing.pairs) {
    CSC_HIP(hipEventSynchronize(p.second));
    float t = 0.f;
    CSC_HIP(hipEventElapsedTime(&t, p.first, p.second));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = g_timing.launches;
  if (bytes) *bytes = g_timing.bytes;
  return CSC_OK;
}

csc_status csc_gather_probe(const int32_t* rowptr, const int32_t* colidx, int64_t n_rows,
                            const void* table, int row_bytes, uint32_t* out, void* stream) {
  return run_gather_probe(rowptr, colidx, n_rows, table, row_bytes, out, as_stream(stream));
}

csc_status csc_autotune(csc_graph h, int w, csc_dtype iter_dt, void* work, size_t work_bytes,
                        void* stream, int* variant) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "bad iterate type");
  Graph& g = h->g;
  hipStream_t s = as_stream(stream);
  const size_t need = filter_workspace(g.n, w, iter_dt);
  // X and Y for the trial filters sit after the filter workspace
  const size_t xb = align_up(static_cast<size_t>(g.n) * w * sizeof(float));
  if (!work || work_bytes < need + 2 * xb)
    return fail(CSC_E_ARG, "autotune workspace too small: need " + std::to_string(need + 2 * xb));
  char* base = static_cast<char*>(work);
  void* X = base + need;
  void* Y = base + need + xb;
  CSC_TRY(launch_randn(X, CSC_F32, g.n, w, w, 0, 7, 7, 0.1, s));
  const int m = 8;
  std::vector<double> a(m + 1, 0.1);
  hipEvent_t e0, e1;
  CSC_HIP(hipEventCreate(&e0));
  CSC_HIP(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 1e30f;
  for (int v = 0; v < num_variants(); ++v) {
    const StepShape sh = variant_shape(v, iter_dt);
    if (sh.wt() > 2 * std::max(w, 16)) continue;  // mostly padding
    // warm-up, then timed
    CSC_TRY(run_filter(&g, 2.0, m, a.data(), X, CSC_F32, w, Y, CSC_F32, w, w, iter_dt, nullptr,
                       0, work, need, s, v));
    CSC_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r)
      CSC_TRY(run_filter(&g, 2.0, m, a.data(), X, CSC_F32, w, Y, CSC_F32, w, w, iter_dt, nullptr,
                         0, work, need, s, v));
    CSC_HIP(hipEventRecord(e1, s));
    CSC_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    CSC_HIP(hipEventElapsedTime(&t, e0, e1));
    if (t < best_ms) {
      best_ms = t;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (iter_dt != CSC_F32) g.variant_bf16 = best;
  else g.variant_f32 = best;
  if (variant) *variant = best;
  return CSC_OK;
}

csc_status csc_set_variant(csc_graph h, csc_dtype iter_dt, int variant) {
  if (!h) return fail(CSC_E_ARG, "null graph");
  if (variant < -1 || variant >= num_variants()) return fail(CSC_E_ARG, "bad variant");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "bad iterate type");
  if (iter_dt != CSC_F32) h->g.variant_bf16 = variant;
  else h->g.variant_f32 = variant;
  return CSC_OK;
}

}  // extern "C"
