// Dynamic compressive spectral clustering (Algorithm 1, Sec. 4.1): the host drives the
// snapshot logic (column-block ring, eigencount acceptance, one-sided refinement) and every
// array operation runs on the device through the filter, dot, RNG and k-means kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <tuple>
#include <cmath>
#include <string>
#include <vector>

#include "csc_internal.h"

struct csc_dyn_s {
  int64_t n = 0;
  int d = 0, k = 0, m = 0, qd = 0;
  double p = 0.0;
  csc_damping damp = CSC_DAMP_JACKSON;
  csc_dtype feat_dt = CSC_F32;
  uint64_t seed = 0;
  double lmax = 0.0, tau = 0.0;  // lmax 0: each snapshot uses its graph's spectrum bound
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
  void* basis = nullptr;      // batch x (m + 1) iterate slots of the fresh blocks, or null
  size_t basis_bytes = 0;     // per snapshot
  int batch = 1;              // snapshots whose recurrences advance together
  int nbuf = 1;               // 2: two batches of slots, so the next batch's recurrence runs
                              // on `fs` while the current batch's k-means runs on the caller's
                              // stream
  bool use_graph = false;     // replay the recurrence launches from a captured HIP graph
  hipStream_t cap = nullptr;
  hipStream_t fs = nullptr;
  hipEvent_t ev_start = nullptr, ev_basis[2] = {}, ev_free[2] = {};
  hipGraphExec_t exec[2] = {};
  const void* exec_key[2][10] = {};
  double exec_lmax[2][8] = {};
  void* aux = nullptr;
  size_t aux_bytes = 0;
  // one-pass batches (batch > 1 without kept iterates), two buffers of `batch` slots each:
  // every slot has a filter workspace, a staged n x qd output block, its coefficients and
  // its moments on the device
  bool onepass = false;
  void* owork = nullptr;
  size_t owork_bytes = 0;     // per slot
  void* ostage = nullptr;
  double* ocoef = nullptr;    // 2 batch (m + 1)
  double* omom = nullptr;     // 2 batch (m + 1)
  std::vector<double> ocoef_h;  // host sources of the coefficient uploads, one row per slot
  int variant = 0;
  int t = 0;
  double lam = 0.0;
  int cursor = 0;             // first column of Theta the next fresh block replaces
  void* wrap = nullptr;       // n x qd staging of a fresh block that wraps past column d
  // similarity of consecutive snapshots (Sec. 4 metrics) and the refresh rule
  bool track = false;
  int sim_probes = 0;
  double budget = 0.0;
  csc::Graph pg{};            // device copy of the previous snapshot's operator
  bool have_prev = false;
  float* simbuf = nullptr;    // n x sim_probes: h^{t-1}(L_{t-1}) applied to the first probes
  double* simd = nullptr;     // device: [0] ||dL||_F^2, [1..3] <Y,Y>, <Y,Yp>, <Yp,Yp>
  void* simwork = nullptr;
  size_t simwork_bytes = 0;
  std::vector<double> hist;   // per snapshot: rho_edge, rho_hat, refreshed
};

namespace csc {

namespace {

constexpr uint64_t kSignals = 1;
constexpr uint64_t kKmeans = 2;
uint64_t stream_id(int t, uint64_t purpose) { return 16ull * static_cast<uint64_t>(t) + purpose; }

void free_dyn(csc_dyn st) {
  if (!st) return;
  for (void* p : {st->theta, st->sig, static_cast<void*>(st->C), static_cast<void*>(st->prev),
                  static_cast<void*>(st->scal), st->fwork, st->kwork, st->dwork, st->basis, st->aux,
                  st->owork, st->ostage, static_cast<void*>(st->ocoef), static_cast<void*>(st->omom),
                  st->wrap, static_cast<void*>(st->simbuf), static_cast<void*>(st->simd),
                  st->simwork, static_cast<void*>(st->pg.rowptr), static_cast<void*>(st->pg.colidx),
                  st->pg.vals, static_cast<void*>(st->pg.diag), static_cast<void*>(st->pg.deg)})
    if (p) (void)hipFree(p);
  for (int b = 0; b < 2; ++b) {
    if (st->exec[b]) (void)hipGraphExecDestroy(st->exec[b]);
    if (st->ev_basis[b]) (void)hipEventDestroy(st->ev_basis[b]);
    if (st->ev_free[b]) (void)hipEventDestroy(st->ev_free[b]);
  }
  if (st->ev_start) (void)hipEventDestroy(st->ev_start);
  if (st->cap) (void)hipStreamDestroy(st->cap);
  if (st->fs) (void)hipStreamDestroy(st->fs);
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
  if (qd < 1 || qd > d) return fail(CSC_E_ARG, "need 1 <= (1 - p) d <= d");
  auto* st = new csc_dyn_s();
  st->n = n;
  st->d = d;
  st->k = k;
  st->m = m;
  st->p = p;
  st->qd = qd;
  st->damp = damp;
  st->feat_dt = feat_dt;
  st->seed = seed;
  if (opts) {
    st->batch = opts->batch >= 1 ? opts->batch : 1;
    st->use_graph = opts->use_graph != 0;
    st->lmax = opts->lmax > 0.0 ? opts->lmax : 0.0;  // 0: each graph's own bound
    st->tau = opts->tau;
    st->n_cand = opts->n_cand > 0 ? opts->n_cand : 16;
    st->lloyd = opts->lloyd_iters >= 0 ? opts->lloyd_iters : 20;
    st->init = opts->init;
    st->iter_dt = opts->iter_dt;
    st->sim_probes = opts->sim_probes;
    st->budget = opts->refresh_budget;
    st->track = opts->track_similarity != 0 || opts->sim_probes > 0 || opts->refresh_budget > 0.0;
  }
  if (st->sim_probes < 0 || st->sim_probes > qd || (st->budget > 0.0 && st->sim_probes == 0)) {
    delete st;
    return fail(CSC_E_ARG, "need 0 <= sim_probes <= (1 - p) d, and sim_probes > 0 for a refresh budget");
  }
  if (st->tau <= 0.0) st->tau = std::max(0.5, 2.0 * std::sqrt(2.0 * k / qd));
  if (!iter_type_ok(st->iter_dt)) {
    delete st;
    return fail(CSC_E_DTYPE, "iterates must be F32, BF16 or BF16S");
  }
  if (st->batch > 8) {
    delete st;
    return fail(CSC_E_ARG, "batch must be in [1, 8]");
  }
  if (opts && opts->variant >= num_variants()) {
    delete st;
    return fail(CSC_E_ARG, "variant must be -1 or in [0, " + std::to_string(num_variants()) + ")");
  }
  const size_t es = dtype_size(feat_dt);
  st->fwork_bytes = filter_workspace(n, d, st->iter_dt, m);  // moments up to degree m
  st->kwork_bytes = kmeans_workspace(n, d, k);
  st->dwork_bytes = dot_workspace(n);
  bool ok = hipMalloc(&st->theta, es * n * d) == hipSuccess &&
            hipMalloc(&st->sig, es * n * std::max(d, 2 * st->batch * qd)) == hipSuccess &&
            hipMalloc(&st->C, sizeof(float) * k * d) == hipSuccess &&
            hipMalloc(&st->prev, sizeof(int32_t) * n) == hipSuccess &&
            hipMalloc(&st->scal, sizeof(double) * (m + 2)) == hipSuccess &&
            hipMalloc(&st->fwork, st->fwork_bytes) == hipSuccess &&
            hipMalloc(&st->kwork, st->kwork_bytes) == hipSuccess &&
            hipMalloc(&st->dwork, st->dwork_bytes) == hipSuccess &&
            (d % qd == 0 || hipMalloc(&st->wrap, es * n * qd) == hipSuccess);
  if (ok && st->track) {
    st->simwork_bytes = distance_workspace(n);
    ok = hipMalloc(&st->simd, 4 * sizeof(double)) == hipSuccess &&
         hipMalloc(&st->simwork, st->simwork_bytes) == hipSuccess &&
         (st->sim_probes == 0 ||
          hipMalloc(&st->simbuf, sizeof(float) * n * st->sim_probes) == hipSuccess);
  }
  if (!ok) {
    free_dyn(st);
    return fail(CSC_E_NOMEM, "device allocation failed in csc_dyn_create");
  }
  // Keep all m + 1 iterates of the fresh block when they fit: a refinement of the cut-off is
  // then a new linear combination of stored iterates instead of a second recurrence.
  const int keep = opts ? opts->keep_iterates : -1;
  if (keep == 1 && m + 1 > 256) {
    free_dyn(st);
    return fail(CSC_E_ARG, "keeping the iterates needs m < 256");
  }
  if (keep != 0 && m + 1 <= 256) {
    Graph probe{};
    probe.variant_f32 = probe.variant_bf16 = -1;
    st->variant = (opts && opts->variant >= 0) ? opts->variant : default_variant(&probe, qd, st->iter_dt);
    st->basis_bytes = basis_bytes(n, qd, m, st->iter_dt, st->variant);
    st->aux_bytes = basis_aux_bytes(n, qd, m, st->iter_dt, st->variant);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const size_t margin = size_t(4) << 30;
    const size_t want = st->basis_bytes * st->batch;
    // a second set of slots when it fits, batched or not: the next recurrence then runs
    // beside this one's recombination, refinement and k-means
    if (2 * want + st->aux_bytes + margin <= free_b &&
        hipMalloc(&st->basis, 2 * want) == hipSuccess) {
      st->nbuf = 2;
      if (hipMalloc(&st->aux, st->aux_bytes) != hipSuccess) {
        free_dyn(st);
        return fail(CSC_E_NOMEM, "cannot allocate the basis scratch");
      }
    } else if (keep == 1 || want + st->aux_bytes + margin <= free_b) {
      if (hipMalloc(&st->basis, want) != hipSuccess ||
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
  if (st->batch > 1 && !st->basis) {
    // one-pass batches: the fresh blocks of a batch are filtered together at the cut-off in
    // force when the batch starts, with their moments; a snapshot whose cut-off ends up
    // different is filtered again (all such snapshots of a batch together)
    st->onepass = true;
    st->variant = (opts && opts->variant >= 0) ? opts->variant : [&] {
      Graph probe{};
      probe.variant_f32 = probe.variant_bf16 = -1;
      return default_variant(&probe, qd, st->iter_dt);
    }();
    st->owork_bytes = align_up(make_plan(n, qd, st->iter_dt, st->variant, m).total);
    const size_t slots = 2 * static_cast<size_t>(st->batch);
    st->ocoef_h.assign(slots * (m + 1), 0.0);
    if (hipMalloc(&st->owork, slots * st->owork_bytes) != hipSuccess ||
        hipMalloc(&st->ostage, slots * es * n * qd) != hipSuccess ||
        hipMalloc(&st->ocoef, slots * (m + 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&st->omom, slots * (m + 1) * sizeof(double)) != hipSuccess) {
      free_dyn(st);
      return fail(CSC_E_NOMEM, "cannot allocate the one-pass batch buffers");
    }
  }
  if (st->use_graph && hipStreamCreate(&st->cap) != hipSuccess) {
    free_dyn(st);
    return fail(CSC_E_HIP, "cannot create the capture stream");
  }
  if (st->nbuf == 2 || (st->basis && st->batch == 1) || st->onepass) {
    // non-blocking: callers often work on the null stream, which would otherwise serialise
    // with it; the order between the two streams comes only from the events below
    bool ev_ok = hipStreamCreateWithFlags(&st->fs, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&st->ev_start, hipEventDisableTiming) == hipSuccess;
    for (int b = 0; b < 2 && ev_ok; ++b)
      ev_ok = hipEventCreateWithFlags(&st->ev_basis[b], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&st->ev_free[b], hipEventDisableTiming) == hipSuccess;
    if (!ev_ok) {
      free_dyn(st);
      return fail(CSC_E_HIP, "cannot create the recurrence stream and its events");
    }
  }
  *out = st;
  return CSC_OK;
}

namespace {

// Fresh signals of snapshot t into signal slot `slot`.
csc_status draw_signals(csc_dyn st, int t, int slot, hipStream_t s) {
  const double sigma = 1.0 / std::sqrt(static_cast<double>(st->d));
  char* sig = static_cast<char*>(st->sig) + dtype_size(st->feat_dt) * static_cast<size_t>(slot) * st->n * st->qd;
  return launch_randn(sig, st->feat_dt, st->n, st->qd, st->qd, 0, st->seed, stream_id(t, kSignals), sigma, s);
}

void* sig_slot(csc_dyn st, int slot) {
  return static_cast<char*>(st->sig) + dtype_size(st->feat_dt) * static_cast<size_t>(slot) * st->n * st->qd;
}

void* basis_slot(csc_dyn st, int slot) {
  return static_cast<char*>(st->basis) + st->basis_bytes * static_cast<size_t>(slot);
}

// Spectrum bound a snapshot maps onto [-1, 1]: the fixed option, else the graph's own.
double lmax_for(csc_dyn st, const Graph* g) { return st->lmax > 0.0 ? st->lmax : g->lmax_bound; }

// The recurrences of S snapshots (slots buf * batch + 0..S-1), replayed from a captured graph
// when enabled (one cached graph per buffer, re-captured when the graphs change).
csc_status batch_basis(csc_dyn st, const Graph* const* gs, int S, hipStream_t s, int buf = 0) {
  const void* X[8];
  void* B[8];
  for (int i = 0; i < S; ++i) {
    X[i] = sig_slot(st, buf * st->batch + i);
    B[i] = basis_slot(st, buf * st->batch + i);
  }
  if (!st->use_graph)
    return run_basis_batch(gs, S, st->lmax, st->m, X, st->feat_dt, st->qd, st->qd, st->iter_dt,
                           st->variant, B, st->basis_bytes, s, true);
  const void* key[10] = {};
  double lms[8] = {};
  key[0] = reinterpret_cast<const void*>(static_cast<intptr_t>(S));
  for (int i = 0; i < S; ++i) {
    key[1 + i] = gs[i];
    lms[i] = lmax_for(st, gs[i]);  // a graph update may change a combinatorial bound
  }
  hipGraphExec_t& exec = st->exec[buf];
  bool same = exec != nullptr;
  for (int i = 0; i < 10 && same; ++i) same = key[i] == st->exec_key[buf][i];
  for (int i = 0; i < 8 && same; ++i) same = lms[i] == st->exec_lmax[buf][i];
  if (!same) {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    CSC_HIP(hipStreamBeginCapture(st->cap, hipStreamCaptureModeRelaxed));
    const csc_status cs = run_basis_batch(gs, S, st->lmax, st->m, X, st->feat_dt, st->qd, st->qd,
                                          st->iter_dt, st->variant, B, st->basis_bytes, st->cap, false);
    const hipError_t e = hipStreamEndCapture(st->cap, &graph);
    if (cs != CSC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (e != hipSuccess) return fail(CSC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      exec = nullptr;
      return fail(CSC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    for (int i = 0; i < 10; ++i) st->exec_key[buf][i] = key[i];
    for (int i = 0; i < 8; ++i) st->exec_lmax[buf][i] = lms[i];
  }
  timing_begin(s);
  CSC_HIP(hipGraphLaunch(exec, s));
  timing_end(s, st->m, basis_batch_bytes(gs, S, st->m, st->qd, st->iter_dt));
  return CSC_OK;
}

}  // namespace

namespace {

// Device copy of this snapshot's operator, for the similarity of the next one.  The copy
// grows (synchronising) when a snapshot has more entries than it holds.
csc_status keep_prev(csc_dyn st, const Graph* g, hipStream_t s) {
  Graph& p = st->pg;
  const bool comb = g->lap == CSC_LAP_COMBINATORIAL;
  const size_t es = dtype_size(g->val_dt);
  if (!p.rowptr || p.cap < g->nnz || p.val_dt != g->val_dt || (comb && !p.diag)) {
    CSC_HIP(hipStreamSynchronize(s));
    for (void* q : {static_cast<void*>(p.rowptr), static_cast<void*>(p.colidx), p.vals,
                    static_cast<void*>(p.diag), static_cast<void*>(p.deg)})
      if (q) (void)hipFree(q);
    p = Graph{};
    p.cap = std::max<int64_t>(g->cap, 1);
    p.val_dt = g->val_dt;
    const bool ok = hipMalloc(&p.rowptr, sizeof(int32_t) * (g->n + 1)) == hipSuccess &&
                    hipMalloc(&p.colidx, sizeof(int32_t) * p.cap) == hipSuccess &&
                    hipMalloc(&p.vals, es * p.cap) == hipSuccess &&
                    (!comb || (hipMalloc(&p.diag, sizeof(float) * g->n) == hipSuccess &&
                               hipMalloc(&p.deg, sizeof(double) * g->n) == hipSuccess));
    if (!ok) return fail(CSC_E_NOMEM, "cannot allocate the copy of the previous snapshot");
  }
  CSC_HIP(hipMemcpyAsync(p.rowptr, g->rowptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToDevice, s));
  if (g->nnz > 0) {
    CSC_HIP(hipMemcpyAsync(p.colidx, g->colidx, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice, s));
    CSC_HIP(hipMemcpyAsync(p.vals, g->vals, es * g->nnz, hipMemcpyDeviceToDevice, s));
  }
  if (comb) {
    CSC_HIP(hipMemcpyAsync(p.diag, g->diag, sizeof(float) * g->n, hipMemcpyDeviceToDevice, s));
    CSC_HIP(hipMemcpyAsync(p.deg, g->deg, sizeof(double) * g->n, hipMemcpyDeviceToDevice, s));
  }
  p.n = g->n;
  p.nnz = g->nnz;
  p.lap = g->lap;
  p.lmax_bound = g->lmax_bound;
  p.variant_f32 = g->variant_f32;
  p.variant_bf16 = g->variant_bf16;
  st->have_prev = true;
  return CSC_OK;
}

// Static CSC on snapshot t (Algorithm 1 steps 1-2, and the refresh): d signals from the
// snapshot's stream, their moments as eigencount probes, a dichotomy on [0, lm], the filter
// of all d columns at the found cut-off into Theta; the ring restarts.
csc_status static_pass(csc_dyn st, const Graph* g, double lm, int t, double* cnt, hipStream_t s) {
  const double sigma = 1.0 / std::sqrt(static_cast<double>(st->d));
  std::vector<double> a(st->m + 1), mu(st->m + 1);
  double* mu_d = st->scal + 1;
  CSC_TRY(launch_randn(st->sig, st->feat_dt, st->n, st->d, st->d, 0, st->seed,
                       stream_id(t, kSignals), sigma, s));
  CSC_TRY(run_filter(g, lm, st->m, nullptr, st->sig, st->feat_dt, st->d, nullptr, CSC_F32,
                     0, st->d, st->iter_dt, mu_d, 1, st->fwork, st->fwork_bytes, s));
  CSC_HIP(hipMemcpyAsync(mu.data(), mu_d, sizeof(double) * (st->m + 1), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  bisect_moments(mu.data(), st->m, lm, st->damp, sigma * sigma, st->d, st->k, st->n_cand, 0.0,
                 lm, &st->lam, cnt, nullptr);
  cheb_coeffs(st->m, lm, st->lam, st->damp, a.data());
  CSC_TRY(run_filter(g, lm, st->m, a.data(), st->sig, st->feat_dt, st->d, st->theta,
                     st->feat_dt, st->d, st->d, st->iter_dt, nullptr, 0, st->fwork,
                     st->fwork_bytes, s));
  st->cursor = 0;
  return CSC_OK;
}

csc_status cluster(csc_dyn st, int t, int32_t* labels, hipStream_t s);

// One snapshot of Algorithm 1.  For t >= 2 the fresh signals and (when kept) their iterates
// live in slot `slot`; with pre_basis the signals are drawn and the iterates computed already
// (batched recurrence).
csc_status step_impl(csc_dyn st, const Graph* g, int slot, bool pre_basis, int32_t* labels,
                     double* lambda_t, int* refined, double* count, hipStream_t s,
                     const std::function<csc_status()>& before_kmeans = {}) {
  const int t = ++st->t;
  const double sigma = 1.0 / std::sqrt(static_cast<double>(st->d));
  const double sigma2 = sigma * sigma;
  const size_t es = dtype_size(st->feat_dt);
  std::vector<double> a(st->m + 1), mu(st->m + 1);
  double cnt = 0.0;
  int ref = 0;
  double* mu_d = st->scal + 1;
  const double lm = lmax_for(st, g);

  double rho_e = -1.0, rho_h = -1.0;
  bool refresh = false;
  if (t == 1) {
    // Algorithm 1, steps 1-2: static CSC on G_1 with the d signals as eigencount probes.
    CSC_TRY(static_pass(st, g, lm, t, &cnt, s));
    ref = 1;
  } else {
    // Steps 4-7: fresh q d columns filtered with h^{t-1}, eigencount, optional refinement.
    // the fresh block replaces columns cursor .. cursor + qd - 1 (mod d) of Theta; a block
    // that wraps past the last column is written to a staging buffer and copied in two parts
    const int c0 = st->cursor;
    const bool wraps = c0 + st->qd > st->d;
    char* blk = wraps ? static_cast<char*>(st->wrap)
                      : static_cast<char*>(st->theta) + es * static_cast<size_t>(c0);
    const int64_t ldb = wraps ? st->qd : st->d;
    void* sig = sig_slot(st, slot);
    void* basis = st->basis ? basis_slot(st, slot) : nullptr;
    if (!pre_basis) CSC_TRY(draw_signals(st, t, slot, s));
    cheb_coeffs(st->m, lm, st->lam, st->damp, a.data());
    const bool kept = st->basis != nullptr;
    if (kept) {
      if (!pre_basis) CSC_TRY(batch_basis(st, &g, 1, s));
      CSC_TRY(run_combine(basis, st->n, st->qd, st->m, st->iter_dt, st->variant, a.data(), blk,
                          st->feat_dt, ldb, sig, st->feat_dt, st->qd, st->scal, st->aux,
                          st->aux_bytes, s));
    } else {
      CSC_TRY(run_filter(g, lm, st->m, a.data(), sig, st->feat_dt, st->qd, blk,
                         st->feat_dt, ldb, st->qd, st->iter_dt, nullptr, 0, st->fwork,
                         st->fwork_bytes, s));
      CSC_TRY(launch_dot(sig, st->feat_dt, st->qd, blk, st->feat_dt, ldb, st->n, st->qd,
                         st->scal, st->dwork, st->dwork_bytes, s));
    }
    double dot = 0.0;
    CSC_HIP(hipMemcpyAsync(&dot, st->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    cnt = dot / (sigma2 * st->qd);
    if (st->track && st->have_prev && st->pg.n == g->n && st->pg.lap == g->lap) {
      // Sec. 4 metrics against G_{t-1}: ||L_t - L_{t-1}||_F, and the spectral distance
      // estimated from the first s fresh signals filtered with h^{t-1} on both graphs
      CSC_TRY(graph_distance2(&st->pg, g, st->simd, st->simwork, st->simwork_bytes, s));
      const int sp = st->sim_probes;
      if (sp > 0) {
        const double lmp = lmax_for(st, &st->pg);
        std::vector<double> ap(st->m + 1);
        cheb_coeffs(st->m, lmp, std::min(st->lam, lmp), st->damp, ap.data());
        CSC_TRY(run_filter(&st->pg, lmp, st->m, ap.data(), sig, st->feat_dt, st->qd, st->simbuf,
                           CSC_F32, sp, sp, st->iter_dt, nullptr, 0, st->fwork, st->fwork_bytes, s));
        CSC_TRY(launch_dot(blk, st->feat_dt, ldb, blk, st->feat_dt, ldb, st->n, sp, st->simd + 1,
                           st->dwork, st->dwork_bytes, s));
        CSC_TRY(launch_dot(blk, st->feat_dt, ldb, st->simbuf, CSC_F32, sp, st->n, sp, st->simd + 2,
                           st->dwork, st->dwork_bytes, s));
        CSC_TRY(launch_dot(st->simbuf, CSC_F32, sp, st->simbuf, CSC_F32, sp, st->n, sp, st->simd + 3,
                           st->dwork, st->dwork_bytes, s));
      }
      double v[4] = {};
      CSC_HIP(hipMemcpyAsync(v, st->simd, sizeof(v), hipMemcpyDeviceToHost, s));
      CSC_HIP(hipStreamSynchronize(s));
      rho_e = std::sqrt(std::max(0.0, v[0]));
      if (sp > 0) rho_h = std::sqrt(std::max(0.0, v[1] - 2.0 * v[2] + v[3]) / (sigma2 * sp));
      // Thm 4.1: reusing a fraction p adds about p * rho to the cost bound
      refresh = st->budget > 0.0 && rho_h >= 0.0 && st->p * rho_h > st->budget;
    }
    if (refresh) {
      CSC_TRY(static_pass(st, g, lm, t, &cnt, s));
      ref = 1;
    } else {
      if (std::fabs(cnt - st->k) > st->tau) {
        if (kept)
          CSC_TRY(run_basis_moments(basis, st->n, st->qd, st->m, st->iter_dt, st->variant, mu_d,
                                    st->aux, st->aux_bytes, s));
        else
          CSC_TRY(run_filter(g, lm, st->m, nullptr, sig, st->feat_dt, st->qd, nullptr,
                             CSC_F32, 0, st->qd, st->iter_dt, mu_d, 1, st->fwork, st->fwork_bytes, s));
        CSC_HIP(hipMemcpyAsync(mu.data(), mu_d, sizeof(double) * (st->m + 1), hipMemcpyDeviceToHost, s));
        CSC_HIP(hipStreamSynchronize(s));
        const double prev = std::min(st->lam, lm);  // a combinatorial bound may shrink
        const double lo = cnt < st->k ? prev : 0.0;
        const double hi = cnt < st->k ? lm : prev;
        bisect_moments(mu.data(), st->m, lm, st->damp, sigma2, st->qd, st->k, st->n_cand, lo,
                       hi, &st->lam, &cnt, nullptr);
        cheb_coeffs(st->m, lm, st->lam, st->damp, a.data());
        if (kept)
          CSC_TRY(run_combine(basis, st->n, st->qd, st->m, st->iter_dt, st->variant, a.data(), blk,
                              st->feat_dt, ldb, nullptr, st->feat_dt, 0, nullptr, st->aux,
                              st->aux_bytes, s));
        else
          CSC_TRY(run_filter(g, lm, st->m, a.data(), sig, st->feat_dt, st->qd, blk,
                             st->feat_dt, ldb, st->qd, st->iter_dt, nullptr, 0, st->fwork,
                             st->fwork_bytes, s));
        ref = 1;
      }
      if (wraps) {
        const int first = st->d - c0;  // columns c0 .. d-1, then 0 .. qd - first - 1
        char* th = static_cast<char*>(st->theta);
        CSC_HIP(hipMemcpy2DAsync(th + es * static_cast<size_t>(c0), es * st->d, blk, es * st->qd,
                                 es * first, st->n, hipMemcpyDeviceToDevice, s));
        CSC_HIP(hipMemcpy2DAsync(th, es * st->d, blk + es * static_cast<size_t>(first), es * st->qd,
                                 es * (st->qd - first), st->n, hipMemcpyDeviceToDevice, s));
      }
      st->cursor = (c0 + st->qd) % st->d;
    }
  }
  if (st->track) {
    CSC_TRY(keep_prev(st, g, s));
    st->hist.resize(3 * static_cast<size_t>(t), -1.0);
    st->hist[3 * (t - 1)] = rho_e;
    st->hist[3 * (t - 1) + 1] = rho_h;
    st->hist[3 * (t - 1) + 2] = refresh ? 1.0 : 0.0;
  }

  // the kept iterates and signals of this snapshot are no longer needed: a caller may start
  // the next snapshot's recurrence here, beside the k-means
  if (before_kmeans) CSC_TRY(before_kmeans());
  CSC_TRY(cluster(st, t, labels, s));
  if (lambda_t) *lambda_t = st->lam;
  if (refined) *refined = ref;
  if (count) *count = cnt;
  return CSC_OK;
}

// Step 8 of Algorithm 1: k-means on Theta_t (synchronising).
csc_status cluster(csc_dyn st, int t, int32_t* labels, hipStream_t s) {
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
  return CSC_OK;
}


// ---- one-pass batches ------------------------------------------------------------------

void* stage_slot(csc_dyn st, int slot) {
  return static_cast<char*>(st->ostage) + dtype_size(st->feat_dt) * static_cast<size_t>(slot) * st->n * st->qd;
}
void* owork_slot(csc_dyn st, int slot) { return static_cast<char*>(st->owork) + st->owork_bytes * static_cast<size_t>(slot); }
double* ocoef_slot(csc_dyn st, int slot) { return st->ocoef + static_cast<size_t>(slot) * (st->m + 1); }
double* omom_slot(csc_dyn st, int slot) { return st->omom + static_cast<size_t>(slot) * (st->m + 1); }

// Uploads the coefficients of the step at lam for slot `slot` (graph g's spectrum bound).
csc_status upload_coefs(csc_dyn st, const Graph* g, int slot, double lam, hipStream_t s) {
  double* h = st->ocoef_h.data() + static_cast<size_t>(slot) * (st->m + 1);
  cheb_coeffs(st->m, lmax_for(st, g), lam, st->damp, h);
  CSC_HIP(hipMemcpyAsync(ocoef_slot(st, slot), h, sizeof(double) * (st->m + 1), hipMemcpyHostToDevice, s));
  return CSC_OK;
}

// The one-pass recurrences of the given slots (graphs gs), with moments when asked; replayed
// from a captured graph when enabled and `cached` (the launches read their coefficients
// from the device, so a replay stays valid after new uploads).
csc_status onepass_batch(csc_dyn st, const Graph* const* gs, const int* slots, int S, bool moments,
                         hipStream_t s, int buf, bool cached) {
  const void* X[8];
  void* Y[8];
  void* W[8];
  const double* A[8];
  double* M[8];
  for (int i = 0; i < S; ++i) {
    X[i] = sig_slot(st, slots[i]);
    Y[i] = stage_slot(st, slots[i]);
    W[i] = owork_slot(st, slots[i]);
    A[i] = ocoef_slot(st, slots[i]);
    M[i] = moments ? omom_slot(st, slots[i]) : nullptr;
  }
  auto run = [&](hipStream_t q, bool timed) {
    return run_filter_batch(gs, S, st->lmax, st->m, A, X, st->feat_dt, st->qd, Y, st->feat_dt,
                            st->qd, st->qd, st->iter_dt, st->variant, moments ? M : nullptr, W,
                            st->owork_bytes, q, timed);
  };
  if (!st->use_graph || !cached) return run(s, true);
  const void* key[10] = {};
  double lms[8] = {};
  key[0] = reinterpret_cast<const void*>(static_cast<intptr_t>(S));
  for (int i = 0; i < S; ++i) {
    key[1 + i] = gs[i];
    lms[i] = lmax_for(st, gs[i]);
  }
  hipGraphExec_t& exec = st->exec[buf];
  bool same = exec != nullptr;
  for (int i = 0; i < 10 && same; ++i) same = key[i] == st->exec_key[buf][i];
  for (int i = 0; i < 8 && same; ++i) same = lms[i] == st->exec_lmax[buf][i];
  if (!same) {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    CSC_HIP(hipStreamBeginCapture(st->cap, hipStreamCaptureModeRelaxed));
    const csc_status cs = run(st->cap, false);
    const hipError_t e = hipStreamEndCapture(st->cap, &graph);
    if (cs != CSC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (e != hipSuccess) return fail(CSC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      exec = nullptr;
      return fail(CSC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    for (int i = 0; i < 10; ++i) st->exec_key[buf][i] = key[i];
    for (int i = 0; i < 8; ++i) st->exec_lmax[buf][i] = lms[i];
  }
  timing_begin(s);
  CSC_HIP(hipGraphLaunch(exec, s));
  timing_end(s, st->m, filter_batch_bytes(gs, S, st->m, st->qd, st->iter_dt, true, st->feat_dt));
  return CSC_OK;
}

// Copies a staged n x qd block into Theta at the ring's cursor (two parts when it wraps past
// column d) and advances the cursor.
csc_status place_block(csc_dyn st, const void* blk, hipStream_t s) {
  const size_t es = dtype_size(st->feat_dt);
  const int c0 = st->cursor;
  const int first = std::min(st->qd, st->d - c0);
  char* th = static_cast<char*>(st->theta);
  const char* b = static_cast<const char*>(blk);
  CSC_HIP(hipMemcpy2DAsync(th + es * static_cast<size_t>(c0), es * st->d, b, es * st->qd, es * first,
                           st->n, hipMemcpyDeviceToDevice, s));
  if (first < st->qd)
    CSC_HIP(hipMemcpy2DAsync(th, es * st->d, b + es * static_cast<size_t>(first), es * st->qd,
                             es * (st->qd - first), st->n, hipMemcpyDeviceToDevice, s));
  st->cursor = (c0 + st->qd) % st->d;
  return CSC_OK;
}

// Snapshots i0 .. S-1 (all after the first) in one-pass batches.  Batch b's fresh blocks are
// filtered together at the cut-off in force when it is issued, with their moments.  Its
// snapshots are then decided in order on the host from their moments (Algorithm 1 steps
// 6-7: the count at the current cut-off, and when it misses k by more than tau the one-sided
// dichotomy), which needs no further filtering; the snapshots whose cut-off differs from the
// one they were filtered at are filtered again, together.  The next batch's recurrence is
// then issued on the state's stream, at the updated cut-off, and runs beside this batch's
// k-means.
csc_status steps_onepass(csc_dyn st, const csc_graph* graphs, int i0, int S, int32_t* const* labels,
                         double* lambdas, int* refined, double* counts, hipStream_t s) {
  const int t0 = st->t;
  const int nbatch = (S - i0 + st->batch - 1) / st->batch;
  const double sigma2 = 1.0 / static_cast<double>(st->d);
  hipStream_t fs = st->fs;
  CSC_HIP(hipEventRecord(st->ev_start, s));
  CSC_HIP(hipStreamWaitEvent(fs, st->ev_start, 0));
  double lam_issued[2] = {0.0, 0.0};
  auto range = [&](int b, int* j, int* nb) {
    *j = i0 + b * st->batch;
    *nb = std::min(st->batch, S - *j);
  };
  auto issue = [&](int b) -> csc_status {
    int j, nb;
    range(b, &j, &nb);
    const int buf = b & 1;
    if (b >= 2) CSC_HIP(hipStreamWaitEvent(fs, st->ev_free[buf], 0));
    const Graph* gs[8];
    int slots[8];
    for (int q = 0; q < nb; ++q) {
      gs[q] = &graphs[j + q]->g;
      slots[q] = buf * st->batch + q;
      CSC_TRY(draw_signals(st, t0 + 1 + (j - i0) + q, slots[q], fs));
      CSC_TRY(upload_coefs(st, gs[q], slots[q], st->lam, fs));
    }
    lam_issued[buf] = st->lam;
    CSC_TRY(onepass_batch(st, gs, slots, nb, true, fs, buf, true));
    CSC_HIP(hipEventRecord(st->ev_basis[buf], fs));
    return CSC_OK;
  };
  std::vector<double> mu(static_cast<size_t>(st->batch) * (st->m + 1)), a(st->m + 1);
  CSC_TRY(issue(0));
  for (int b = 0; b < nbatch; ++b) {
    int j, nb;
    range(b, &j, &nb);
    const int buf = b & 1;
    CSC_HIP(hipStreamWaitEvent(s, st->ev_basis[buf], 0));
    CSC_HIP(hipMemcpyAsync(mu.data(), omom_slot(st, buf * st->batch), sizeof(double) * nb * (st->m + 1),
                           hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    // decisions, snapshot by snapshot
    double lam_q[8], cnt_q[8];
    int ref_q[8];
    const Graph* again[8];
    int again_slots[8], n_again = 0;
    for (int q = 0; q < nb; ++q) {
      const Graph* g = &graphs[j + q]->g;
      const double lm = lmax_for(st, g);
      const double* m_q = mu.data() + static_cast<size_t>(q) * (st->m + 1);
      cheb_coeffs(st->m, lm, st->lam, st->damp, a.data());
      double c = 0.0;
      for (int i = 0; i <= st->m; ++i) c += a[i] * m_q[i];
      c /= sigma2 * st->qd;
      int ref = 0;
      if (std::fabs(c - st->k) > st->tau) {
        const double prev = std::min(st->lam, lm);
        const double lo = c < st->k ? prev : 0.0;
        const double hi = c < st->k ? lm : prev;
        bisect_moments(m_q, st->m, lm, st->damp, sigma2, st->qd, st->k, st->n_cand, lo, hi,
                       &st->lam, &c, nullptr);
        ref = 1;
      }
      lam_q[q] = st->lam;
      cnt_q[q] = c;
      ref_q[q] = ref;
      if (st->lam != lam_issued[buf]) {
        again[n_again] = g;
        again_slots[n_again] = buf * st->batch + q;
        CSC_TRY(upload_coefs(st, g, again_slots[n_again], st->lam, s));
        ++n_again;
      }
    }
    if (n_again > 0) CSC_TRY(onepass_batch(st, again, again_slots, n_again, false, s, buf, false));
    if (b + 1 < nbatch) {
      // the next batch may start once this batch's filtering is enqueued (its buffer is the
      // other one; that buffer's last use is fenced by ev_free)
      CSC_TRY(issue(b + 1));
    }
    for (int q = 0; q < nb; ++q) {
      const int t = ++st->t;
      CSC_TRY(place_block(st, stage_slot(st, buf * st->batch + q), s));
      CSC_TRY(cluster(st, t, labels[j + q], s));
      if (lambdas) lambdas[j + q] = lam_q[q];
      if (refined) refined[j + q] = ref_q[q];
      if (counts) counts[j + q] = cnt_q[q];
    }
    CSC_HIP(hipEventRecord(st->ev_free[buf], s));
  }
  return CSC_OK;
}
}  // namespace

csc_status dyn_step(csc_dyn st, csc_graph gh, int32_t* labels, double* lambda_t, int* refined,
                    double* count, void* stream) {
  if (!st || !gh || !labels) return fail(CSC_E_ARG, "null argument");
  if (gh->g.n != st->n) return fail(CSC_E_ARG, "graph size differs from the state's");
  return step_impl(st, &gh->g, 0, false, labels, lambda_t, refined, count, as_stream(stream));
}

// S snapshots in order.  After the first snapshot of the sequence, the fresh blocks of up to
// `batch` snapshots are drawn and their recurrences advanced together (one launch per step);
// the cut-off decisions, refinements and k-means then run snapshot by snapshot as in
// Algorithm 1, so the results equal those of S calls to dyn_step.  The recurrences do not
// depend on earlier snapshots' results, so with two buffers the next batch's recurrence is
// issued on the state's own stream before the current batch's decisions and k-means run on
// the caller's stream; events order the buffers' reuse.
csc_status dyn_steps(csc_dyn st, const csc_graph* graphs, int S, int32_t* const* labels,
                     double* lambdas, int* refined, double* counts, void* stream) {
  if (!st || !graphs || !labels || S < 0) return fail(CSC_E_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  for (int i = 0; i < S; ++i) {
    if (!graphs[i] || !labels[i]) return fail(CSC_E_ARG, "null graph or labels");
    if (graphs[i]->g.n != st->n) return fail(CSC_E_ARG, "graph size differs from the state's");
  }
  int i = 0;
  auto out = [&](int j) {
    return std::make_tuple(lambdas ? lambdas + j : nullptr, refined ? refined + j : nullptr,
                           counts ? counts + j : nullptr);
  };
  // the first snapshot, no kept iterates and no one-pass batches, or similarity tracking:
  // one at a time
  while (i < S && (st->t == 0 || (!st->basis && !st->onepass) || st->track)) {
    auto [l, r, c] = out(i);
    CSC_TRY(step_impl(st, &graphs[i]->g, 0, false, labels[i], l, r, c, s));
    ++i;
  }
  if (i >= S) return CSC_OK;
  if (st->onepass) {
    const csc_status rc = steps_onepass(st, graphs, i, S, labels, lambdas, refined, counts, s);
    if (rc != CSC_OK) (void)hipStreamSynchronize(st->fs);
    return rc;
  }
  const int i0 = i;
  const int t0 = st->t;  // snapshot i has index t0 + 1 + (i - i0)
  const int nbatch = (S - i0 + st->batch - 1) / st->batch;
  const bool pipe = st->nbuf == 2;
  // one buffer of kept iterates, one snapshot per batch: the next snapshot's recurrence starts
  // on the state's stream as soon as this snapshot's recombination and refinement are done,
  // and runs beside its k-means
  const bool early = !pipe && st->batch == 1 && st->fs != nullptr;
  hipStream_t fs = (pipe || early) ? st->fs : s;
  if (pipe || early) {
    // the recurrence stream sees everything the caller enqueued before (graph updates)
    CSC_HIP(hipEventRecord(st->ev_start, s));
    CSC_HIP(hipStreamWaitEvent(fs, st->ev_start, 0));
  }
  auto issue = [&](int b) -> csc_status {
    const int j = i0 + b * st->batch;
    const int nb = std::min(st->batch, S - j);
    const int buf = pipe ? (b & 1) : 0;
    if (pipe && b >= 2) CSC_HIP(hipStreamWaitEvent(fs, st->ev_free[buf], 0));
    const Graph* gs[8];
    for (int q = 0; q < nb; ++q) {
      gs[q] = &graphs[j + q]->g;
      CSC_TRY(draw_signals(st, t0 + 1 + (j - i0) + q, buf * st->batch + q, fs));
    }
    CSC_TRY(batch_basis(st, gs, nb, fs, buf));
    if (pipe || early) CSC_HIP(hipEventRecord(st->ev_basis[buf], fs));
    return CSC_OK;
  };
  // on a failure, work already issued on the recurrence stream is drained before returning,
  // so that no later call races with it
  const csc_status rc = [&]() -> csc_status {
    CSC_TRY(issue(0));
    for (int b = 0; b < nbatch; ++b) {
      if (pipe && b + 1 < nbatch) CSC_TRY(issue(b + 1));
      const int j = i0 + b * st->batch;
      const int nb = std::min(st->batch, S - j);
      const int buf = pipe ? (b & 1) : 0;
      if (pipe || early) CSC_HIP(hipStreamWaitEvent(s, st->ev_basis[buf], 0));
      // early: before this snapshot's k-means, the next recurrence waits for the work enqueued
      // so far on the caller's stream (recombination, refinement) and is then issued
      const std::function<csc_status()> next = [&]() -> csc_status {
        CSC_HIP(hipEventRecord(st->ev_free[0], s));
        CSC_HIP(hipStreamWaitEvent(fs, st->ev_free[0], 0));
        return issue(b + 1);
      };
      const bool hand_over = early && b + 1 < nbatch;
      for (int q = 0; q < nb; ++q) {
        auto [l, r, c] = out(j + q);
        CSC_TRY(step_impl(st, &graphs[j + q]->g, buf * st->batch + q, true, labels[j + q], l, r,
                          c, s, hand_over ? next : std::function<csc_status()>()));
      }
      if (pipe) CSC_HIP(hipEventRecord(st->ev_free[buf], s));
      if (!pipe && !early && b + 1 < nbatch) CSC_TRY(issue(b + 1));
    }
    return CSC_OK;
  }();
  if (rc != CSC_OK && fs != s) (void)hipStreamSynchronize(fs);
  return rc;
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

constexpr uint64_t kStateMagic = 0x31304e5944435343ull;

size_t dyn_state_bytes(csc_dyn st) {
  if (!st) return 0;
  return sizeof(csc_dyn_header) + dtype_size(st->feat_dt) * static_cast<size_t>(st->n) * st->d +
         sizeof(float) * static_cast<size_t>(st->k) * st->d + sizeof(int32_t) * static_cast<size_t>(st->n);
}

csc_status dyn_export(csc_dyn st, void* buf, size_t bytes, hipStream_t s) {
  if (!st || !buf) return fail(CSC_E_ARG, "null argument");
  if (st->t < 1) return fail(CSC_E_STATE, "nothing to export before the first snapshot");
  if (bytes < dyn_state_bytes(st)) return fail(CSC_E_ARG, "state buffer too small");
  csc_dyn_header h{};
  h.magic = kStateMagic;
  h.n = st->n;
  h.d = st->d;
  h.k = st->k;
  h.m = st->m;
  h.qd = st->qd;
  h.feat_dt = static_cast<int32_t>(st->feat_dt);
  h.t = st->t;
  h.cursor = st->cursor;
  h.seed = st->seed;
  h.lambda = st->lam;
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t tb = dtype_size(st->feat_dt) * static_cast<size_t>(st->n) * st->d;
  const size_t cb = sizeof(float) * static_cast<size_t>(st->k) * st->d;
  CSC_HIP(hipMemcpyAsync(p, st->theta, tb, hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(p + tb, st->C, cb, hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(p + tb + cb, st->prev, sizeof(int32_t) * st->n, hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  return CSC_OK;
}

csc_status dyn_import(csc_dyn st, const void* buf, size_t bytes, hipStream_t s) {
  if (!st || !buf) return fail(CSC_E_ARG, "null argument");
  if (bytes < dyn_state_bytes(st)) return fail(CSC_E_ARG, "state buffer too small");
  csc_dyn_header h{};
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic) return fail(CSC_E_ARG, "not a dynamic CSC state");
  if (h.n != st->n || h.d != st->d || h.k != st->k || h.m != st->m || h.qd != st->qd ||
      h.feat_dt != static_cast<int32_t>(st->feat_dt) || h.seed != st->seed)
    return fail(CSC_E_ARG, "the state was exported from a handle with other parameters");
  if (h.t < 1 || h.cursor < 0 || h.cursor >= st->d || !(h.lambda >= 0.0))
    return fail(CSC_E_ARG, "corrupt state header");
  const char* p = static_cast<const char*>(buf) + sizeof(h);
  const size_t tb = dtype_size(st->feat_dt) * static_cast<size_t>(st->n) * st->d;
  const size_t cb = sizeof(float) * static_cast<size_t>(st->k) * st->d;
  CSC_HIP(hipMemcpyAsync(st->theta, p, tb, hipMemcpyHostToDevice, s));
  CSC_HIP(hipMemcpyAsync(st->C, p + tb, cb, hipMemcpyHostToDevice, s));
  CSC_HIP(hipMemcpyAsync(st->prev, p + tb + cb, sizeof(int32_t) * st->n, hipMemcpyHostToDevice, s));
  CSC_HIP(hipStreamSynchronize(s));
  st->t = h.t;
  st->cursor = h.cursor;
  st->lam = h.lambda;
  st->have_prev = false;
  if (st->track) st->hist.assign(3 * static_cast<size_t>(h.t), -1.0);
  return CSC_OK;
}

csc_status dyn_similarity(csc_dyn st, int t, double* rho_edge, double* rho_hat, int* refreshed) {
  if (!st) return fail(CSC_E_ARG, "null state");
  if (!st->track) return fail(CSC_E_STATE, "similarity tracking is off for this state");
  if (t < 1 || t > st->t) return fail(CSC_E_ARG, "snapshot index out of range");
  if (rho_edge) *rho_edge = st->hist[3 * (t - 1)];
  if (rho_hat) *rho_hat = st->hist[3 * (t - 1) + 1];
  if (refreshed) *refreshed = st->hist[3 * (t - 1) + 2] > 0.5 ? 1 : 0;
  return CSC_OK;
}

csc_status dyn_destroy(csc_dyn st) {
  free_dyn(st);
  return CSC_OK;
}

}  // namespace csc
