// Dynamic compressive spectral clustering (Algorithm 1, Sec. 4.1): the host drives the
// snapshot logic (column-block ring, eigencount acceptance, one-sided refinement) and every
// array operation runs on the device through the filter, dot, RNG and k-means kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "csc_internal.h"

struct csc_dyn_s {
  int64_t n = 0;
  int d = 0, k = 0, m = 0, qd = 0, nblocks = 0;
  double p = 0.0;
  csc_damping damp = CSC_DAMP_JACKSON;
  csc_dtype feat_dt = CSC_F32;
  uint64_t seed = 0;
  double lmax = 2.0, tau = 0.0;
  int n_cand = 16, lloyd = 20, init = 0;
  csc_dtype iter_dt = CSC_F32;
  void* theta = nullptr;      // n x d, feat_dt
  void* sig = nullptr;        // n x d, feat_dt (fresh signals)
  float* C = nullptr;         // k x d
  int32_t* prev = nullptr;    // n, labels of the previous snapshot
  double* scal = nullptr;     // device scalars: [0] dot, [1 .. m+1] moments
  void* fwork = nullptr;
  size_t fwork_bytes = 0;
  void* kwork = nullptr;
  size_t kwork_bytes = 0;
  void* dwork = nullptr;
  size_t dwork_bytes = 0;
  void* basis = nullptr;      // (m + 1) iterate slots of the fresh block, or null
  size_t basis_bytes = 0;
  void* aux = nullptr;
  size_t aux_bytes = 0;
  int variant = 0;
  int t = 0;
  double lam = 0.0;
  int next_block = 0;
};

namespace csc {

namespace {

constexpr uint64_t kSignals = 1;
constexpr uint64_t kKmeans = 2;
uint64_t stream_id(int t, uint64_t purpose) { return 16ull * static_cast<uint64_t>(t) + purpose; }

void free_dyn(csc_dyn st) {
  if (!st) return;
  for (void* p : {st->theta, st->sig, static_cast<void*>(st->C), static_cast<void*>(st->prev),
                  static_cast<void*>(st->scal), st->fwork, st->kwork, st->dwork, st->basis, st->aux})
    if (p) (void)hipFree(p);
  delete st;
}

__global__ void k_zero_f(float* p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

}  // namespace

csc_status dyn_create(int64_t n, int d, int k, double p, int m, csc_damping damp,
                      csc_dtype feat_dt, uint64_t seed, const csc_dyn_opts* opts, csc_dyn* out) {
  if (!out) return fail(CSC_E_ARG, "out is null");
  *out = nullptr;
  if (n < 1 || d < 1 || d > 256 || k < 1 || k > n || m < 1 || m > 4096)
    return fail(CSC_E_ARG, "need n >= k >= 1, 1 <= d <= 256, 1 <= m <= 4096");
  if (!(p >= 0.0 && p < 1.0)) return fail(CSC_E_ARG, "need 0 <= p < 1");
  if (feat_dt != CSC_F32 && feat_dt != CSC_BF16) return fail(CSC_E_DTYPE, "features must be F32 or BF16");
  const int qd = static_cast<int>(std::lround((1.0 - p) * d));
  if (qd < 1 || d % qd != 0) return fail(CSC_E_ARG, "(1 - p) d must be a positive divisor of d");
  auto* st = new csc_dyn_s();
  st->n = n;
  st->d = d;
  st->k = k;
  st->m = m;
  st->p = p;
  st->qd = qd;
  st->nblocks = d / qd;
  st->damp = damp;
  st->feat_dt = feat_dt;
  st->seed = seed;
  if (opts) {
    st->lmax = opts->lmax > 0.0 ? opts->lmax : 2.0;
    st->tau = opts->tau;
    st->n_cand = opts->n_cand > 0 ? opts->n_cand : 16;
    st->lloyd = opts->lloyd_iters >= 0 ? opts->lloyd_iters : 20;
    st->init = opts->init;
    st->iter_dt = opts->iter_dt;
  }
  if (st->tau <= 0.0) st->tau = std::max(0.5, 2.0 * std::sqrt(2.0 * k / qd));
  if (st->iter_dt != CSC_F32 && st->iter_dt != CSC_BF16) {
    delete st;
    return fail(CSC_E_DTYPE, "iterates must be F32 or BF16");
  }
  const size_t es = dtype_size(feat_dt);
  st->fwork_bytes = filter_workspace(n, d, st->iter_dt);
  st->kwork_bytes = kmeans_workspace(n, d, k);
  st->dwork_bytes = dot_workspace(n);
  bool ok = hipMalloc(&st->theta, es * n * d) == hipSuccess &&
            hipMalloc(&st->sig, es * n * d) == hipSuccess &&
            hipMalloc(&st->C, sizeof(float) * k * d) == hipSuccess &&
            hipMalloc(&st->prev, sizeof(int32_t) * n) == hipSuccess &&
            hipMalloc(&st->scal, sizeof(double) * (m + 2)) == hipSuccess &&
            hipMalloc(&st->fwork, st->fwork_bytes) == hipSuccess &&
            hipMalloc(&st->kwork, st->kwork_bytes) == hipSuccess &&
            hipMalloc(&st->dwork, st->dwork_bytes) == hipSuccess;
  if (!ok) {
    free_dyn(st);
    return fail(CSC_E_NOMEM, "device allocation failed in csc_dyn_create");
  }
  // Keep all m + 1 iterates of the fresh block when they fit: a refinement of the cut-off is
  // then a new linear combination of stored iterates instead of a second recurrence.
  const int keep = opts ? opts->keep_iterates : -1;
  if (keep != 0 && m + 1 <= 512) {
    Graph probe{};
    probe.variant_f32 = probe.variant_bf16 = -1;
    st->variant = default_variant(&probe, qd, st->iter_dt);
    st->basis_bytes = basis_bytes(n, qd, m, st->iter_dt, st->variant);
    st->aux_bytes = basis_aux_bytes(n, m);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const size_t margin = size_t(4) << 30;
    if (keep == 1 || st->basis_bytes + st->aux_bytes + margin <= free_b) {
      if (hipMalloc(&st->basis, st->basis_bytes) != hipSuccess ||
          hipMalloc(&st->aux, st->aux_bytes) != hipSuccess) {
        if (keep == 1) {
          free_dyn(st);
          return fail(CSC_E_NOMEM, "cannot keep the iterates: allocation failed");
        }
        if (st->basis) (void)hipFree(st->basis);
        if (st->aux) (void)hipFree(st->aux);
        st->basis = st->aux = nullptr;
      }
    }
  }
  *out = st;
  return CSC_OK;
}

csc_status dyn_step(csc_dyn st, csc_graph gh, int32_t* labels, double* lambda_t, int* refined,
                    double* count, void* stream) {
  if (!st || !gh || !labels) return fail(CSC_E_ARG, "null argument");
  const Graph* g = &gh->g;
  if (g->n != st->n) return fail(CSC_E_ARG, "graph size differs from the state's");
  hipStream_t s = as_stream(stream);
  const int t = ++st->t;
  const double sigma = 1.0 / std::sqrt(static_cast<double>(st->d));
  const double sigma2 = sigma * sigma;
  const size_t es = dtype_size(st->feat_dt);
  std::vector<double> a(st->m + 1), mu(st->m + 1);
  double cnt = 0.0;
  int ref = 0;
  double* mu_d = st->scal + 1;

  if (t == 1) {
    // Algorithm 1, steps 1-2: static CSC on G_1 with the d signals as eigencount probes.
    CSC_TRY(launch_randn(st->sig, st->feat_dt, st->n, st->d, st->d, 0, st->seed,
                         stream_id(t, kSignals), sigma, s));
    CSC_TRY(run_filter(g, st->lmax, st->m, nullptr, st->sig, st->feat_dt, st->d, nullptr, CSC_F32,
                       0, st->d, st->iter_dt, mu_d, 1, st->fwork, st->fwork_bytes, s));
    CSC_HIP(hipMemcpyAsync(mu.data(), mu_d, sizeof(double) * (st->m + 1), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    bisect_moments(mu.data(), st->m, st->lmax, st->damp, sigma2, st->d, st->k, st->n_cand, 0.0,
                   st->lmax, &st->lam, &cnt, nullptr);
    cheb_coeffs(st->m, st->lmax, st->lam, st->damp, a.data());
    CSC_TRY(run_filter(g, st->lmax, st->m, a.data(), st->sig, st->feat_dt, st->d, st->theta,
                       st->feat_dt, st->d, st->d, st->iter_dt, nullptr, 0, st->fwork,
                       st->fwork_bytes, s));
    st->next_block = 0;
    ref = 1;
  } else {
    // Steps 4-7: fresh q d columns filtered with h^{t-1}, eigencount, optional refinement.
    const int b = st->next_block;
    char* blk = static_cast<char*>(st->theta) + es * static_cast<size_t>(b) * st->qd;
    CSC_TRY(launch_randn(st->sig, st->feat_dt, st->n, st->qd, st->qd, 0, st->seed,
                         stream_id(t, kSignals), sigma, s));
    cheb_coeffs(st->m, st->lmax, st->lam, st->damp, a.data());
    const bool kept = st->basis != nullptr;
    if (kept) {
      CSC_TRY(run_basis(g, st->lmax, st->m, st->sig, st->feat_dt, st->qd, st->qd, st->iter_dt,
                        st->variant, st->basis, st->basis_bytes, s));
      CSC_TRY(run_combine(st->basis, st->n, st->qd, st->m, st->iter_dt, st->variant, a.data(), blk,
                          st->feat_dt, st->d, st->sig, st->feat_dt, st->qd, st->scal, st->aux,
                          st->aux_bytes, s));
    } else {
      CSC_TRY(run_filter(g, st->lmax, st->m, a.data(), st->sig, st->feat_dt, st->qd, blk,
                         st->feat_dt, st->d, st->qd, st->iter_dt, nullptr, 0, st->fwork,
                         st->fwork_bytes, s));
      CSC_TRY(launch_dot(st->sig, st->feat_dt, st->qd, blk, st->feat_dt, st->d, st->n, st->qd,
                         st->scal, st->dwork, st->dwork_bytes, s));
    }
    double dot = 0.0;
    CSC_HIP(hipMemcpyAsync(&dot, st->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    cnt = dot / (sigma2 * st->qd);
    if (std::fabs(cnt - st->k) > st->tau) {
      if (kept)
        CSC_TRY(run_basis_moments(st->basis, st->n, st->qd, st->m, st->iter_dt, st->variant, mu_d,
                                  st->aux, st->aux_bytes, s));
      else
        CSC_TRY(run_filter(g, st->lmax, st->m, nullptr, st->sig, st->feat_dt, st->qd, nullptr,
                           CSC_F32, 0, st->qd, st->iter_dt, mu_d, 1, st->fwork, st->fwork_bytes, s));
      CSC_HIP(hipMemcpyAsync(mu.data(), mu_d, sizeof(double) * (st->m + 1), hipMemcpyDeviceToHost, s));
      CSC_HIP(hipStreamSynchronize(s));
      const double lo = cnt < st->k ? st->lam : 0.0;
      const double hi = cnt < st->k ? st->lmax : st->lam;
      bisect_moments(mu.data(), st->m, st->lmax, st->damp, sigma2, st->qd, st->k, st->n_cand, lo,
                     hi, &st->lam, &cnt, nullptr);
      cheb_coeffs(st->m, st->lmax, st->lam, st->damp, a.data());
      if (kept)
        CSC_TRY(run_combine(st->basis, st->n, st->qd, st->m, st->iter_dt, st->variant, a.data(), blk,
                            st->feat_dt, st->d, nullptr, st->feat_dt, 0, nullptr, st->aux,
                            st->aux_bytes, s));
      else
        CSC_TRY(run_filter(g, st->lmax, st->m, a.data(), st->sig, st->feat_dt, st->qd, blk,
                           st->feat_dt, st->d, st->qd, st->iter_dt, nullptr, 0, st->fwork,
                           st->fwork_bytes, s));
      ref = 1;
    }
    st->next_block = (b + 1) % st->nblocks;
  }

  // Step 8: k-means on Theta_t.
  int init = 0;
  if (st->init == 1 && t > 1) {
    const int64_t kd = static_cast<int64_t>(st->k) * st->d;
    hipLaunchKernelGGL(k_zero_f, dim3(static_cast<unsigned>((kd + 255) / 256)), dim3(256), 0, s,
                       st->C, kd);
    CSC_TRY(launch_kmeans_update(st->theta, st->feat_dt, st->d, st->n, st->d, st->prev, st->k,
                                 st->C, nullptr, st->kwork, st->kwork_bytes, s));
    init = 1;
  }
  CSC_TRY(run_kmeans(st->theta, st->feat_dt, st->d, st->n, st->d, st->k, st->lloyd, init,
                     st->seed, stream_id(t, kKmeans), st->C, labels, nullptr, st->kwork,
                     st->kwork_bytes, s));
  CSC_HIP(hipMemcpyAsync(st->prev, labels, sizeof(int32_t) * st->n, hipMemcpyDeviceToDevice, s));
  CSC_HIP(hipStreamSynchronize(s));
  if (lambda_t) *lambda_t = st->lam;
  if (refined) *refined = ref;
  if (count) *count = cnt;
  return CSC_OK;
}

csc_status dyn_features(csc_dyn st, const void** theta, csc_dtype* dt, int64_t* ld,
                        const float** centroids) {
  if (!st) return fail(CSC_E_ARG, "null state");
  if (theta) *theta = st->theta;
  if (dt) *dt = st->feat_dt;
  if (ld) *ld = st->d;
  if (centroids) *centroids = st->C;
  return CSC_OK;
}

csc_status dyn_destroy(csc_dyn st) {
  free_dyn(st);
  return CSC_OK;
}

}  // namespace csc
