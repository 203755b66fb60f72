// Internal declarations shared by the libcsc translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/csc.h"

namespace csc {

// ------------------------------------------------------------------------------------
// error reporting

void set_error(const std::string& msg);
csc_status fail(csc_status st, const std::string& msg);

#define CSC_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::csc::fail(CSC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

#define CSC_TRY(call)                  \
  do {                                 \
    csc_status s_ = (call);            \
    if (s_ != CSC_OK) return s_;       \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Element size; for the split iterate modes (CSC_BF16S, CSC_F16S), the size of the stored
// (gathered) copy.
inline size_t dtype_size(csc_dtype t) {
  switch (t) {
    case CSC_F32: return 4;
    case CSC_BF16: return 2;
    case CSC_F64: return 8;
    case CSC_BF16S: return 2;
    case CSC_F16: return 2;
    case CSC_F16S: return 2;
  }
  return 0;
}

inline bool iter_type_ok(csc_dtype t) {
  return t == CSC_F32 || t == CSC_BF16 || t == CSC_BF16S || t == CSC_F16 || t == CSC_F16S;
}
// split modes: 16-bit copies for the gathers and the kept basis, FP32 recurrence state
inline bool iter_split(csc_dtype t) { return t == CSC_BF16S || t == CSC_F16S; }
// binary16 copies (CSC_F16, CSC_F16S)
inline bool iter_half(csc_dtype t) { return t == CSC_F16 || t == CSC_F16S; }
// bytes per element of the separate FP32 recurrence state (split modes only)
inline size_t state_size(csc_dtype t) { return iter_split(t) ? 4 : 0; }

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------------------------
// bfloat16 storage: the upper half of an IEEE binary32, rounded to nearest even

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  union { uint32_t u; float f; } v;
  v.u = static_cast<uint32_t>(h) << 16;
  return v.f;
}

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  union { uint32_t u; float f; } v;
  v.f = f;
  if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu)) return 0x7fc0;  // NaN
  uint32_t lsb = (v.u >> 16) & 1u;
  return static_cast<uint16_t>((v.u + 0x7fffu + lsb) >> 16);
}

// ------------------------------------------------------------------------------------
// graph handle

struct Graph {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t cap = 0;
  csc_dtype val_dt = CSC_F32;
  int32_t* rowptr = nullptr;  // n + 1
  int32_t* colidx = nullptr;  // cap
  void* vals = nullptr;       // cap, val_dt
  double* dinv = nullptr;     // n
  csc_laplacian lap = CSC_LAP_NORMALIZED;
  float* diag = nullptr;      // combinatorial only: degrees d_r (the diagonal of L)
  double* deg = nullptr;      // combinatorial only: FP64 degrees, for the spectrum bound
  double lmax_bound = 2.0;    // fixed spectrum bound (host copy)
  int32_t* mirror = nullptr;  // cap
  int32_t* flags = nullptr;   // validation / counters (device, 4 ints)
  int variant_f32 = -1;       // step-kernel shape chosen by the autotuner (-1 = default)
  int variant_bf16 = -1;
  bool mirror_valid = false;
};

csc_status graph_build(Graph* g, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                       const double* w, int validate, hipStream_t s);
csc_status graph_ensure_mirror(Graph* g, hipStream_t s);
// dW (device double[nnz]) from dA (device float[nnz]); q: device double[n] scratch
csc_status graph_weight_grad(Graph* g, const float* dA, double* dW, double* q, hipStream_t s);
// compressive k-means (k_compress.hip)
size_t compressive_workspace(int64_t n, int d, int k, int ns);
csc_status run_compressive(const Graph* g, const void* F, csc_dtype f_dt, int64_t ldf, int d, int k,
                           int ns, int r, double gamma, int lloyd, int cg_iters, double cg_tol,
                           uint64_t seed, uint64_t sample_stream, uint64_t kmeans_stream,
                           int32_t* labels, int32_t* samples, int32_t* sample_labels, float* X,
                           int* iters_done, void* work, size_t work_bytes, hipStream_t st);
// ||L(b) - L(a)||_F^2 into *out (device double); graphs of the same n and Laplacian kind.
size_t distance_workspace(int64_t n);
csc_status graph_distance2(const Graph* a, const Graph* b, double* out, void* work,
                           size_t work_bytes, hipStream_t s);

// ------------------------------------------------------------------------------------
// fused Chebyshev recurrence

// Shape of one step kernel: `lpr` lanes per row, each lane `vec` consecutive columns, so
// one column tile holds wt = lpr * vec columns.
struct StepShape {
  int lpr;
  int vec;
  int wt() const { return lpr * vec; }
};

int num_variants();
StepShape variant_shape(int variant, csc_dtype iter_dt);
int default_variant(const Graph* g, int w, csc_dtype iter_dt);

struct FilterPlan {
  int64_t n;
  int w;          // true number of columns
  int variant;
  StepShape shape;
  int ntiles;
  int wpad;       // ntiles * wt
  csc_dtype iter_dt;
  // workspace carve-up (byte offsets)
  size_t off_z0, off_z1, off_s0, off_s1, off_acc, off_part, off_mom;
  size_t total;
  int64_t rows_per_block;
  int64_t row_blocks;
};

FilterPlan make_plan(int64_t n, int w, csc_dtype iter_dt, int variant, int m_for_moments);
// every variant, moments up to degree m_max (the ABI's filter calls accept m <= 4096)
size_t filter_workspace(int64_t n, int w, csc_dtype iter_dt, int m_max = 4096);

// Runs the whole recurrence.  mode_acc: accumulate Y; moments: device double[m+1] or null.
csc_status run_filter(const Graph* g, double lmax, int m, const double* a, const void* X,
                      csc_dtype x_dt, int64_t ldx, void* Y, csc_dtype y_dt, int64_t ldy,
                      int w, csc_dtype iter_dt, double* moments, int moments_only, void* work,
                      size_t work_bytes, hipStream_t s, int variant_override = -2);

// Stored basis Z_0..Z_m (tiled, one slot per j) and its uses.
size_t basis_bytes(int64_t n, int w, int m, csc_dtype iter_dt, int variant);
size_t basis_aux_bytes(int64_t n, int w, int m, csc_dtype iter_dt, int variant);
csc_status run_basis(const Graph* g, double lmax, int m, const void* X, csc_dtype x_dt, int64_t ldx,
                     int w, csc_dtype iter_dt, int variant, void* basis, size_t bytes, hipStream_t s);
csc_status run_combine(const void* basis, int64_t n, int w, int m, csc_dtype iter_dt, int variant,
                       const double* a, void* Y, csc_dtype y_dt, int64_t ldy, const void* P,
                       csc_dtype p_dt, int64_t ldp, double* dot, void* aux, size_t aux_bytes,
                       hipStream_t s);
csc_status run_basis_moments(const void* basis, int64_t n, int w, int m, csc_dtype iter_dt,
                             int variant, double* moments, void* aux, size_t aux_bytes,
                             hipStream_t s);
// S (<= 8) independent recurrences advanced together, one launch per step.
csc_status run_basis_batch(const Graph* const* graphs, int S, double lmax, int m,
                           const void* const* X, csc_dtype x_dt, int64_t ldx, int w,
                           csc_dtype iter_dt, int variant, void* const* bases, size_t bytes,
                           hipStream_t s, bool timed);
double basis_batch_bytes(const Graph* const* graphs, int S, int m, int w, csc_dtype iter_dt);
// S (<= 8) one-pass filters with per-snapshot device coefficients (and moments), one launch
// per step; work[i] holds make_plan(n, w, iter_dt, variant, m).total bytes.
csc_status run_filter_batch(const Graph* const* graphs, int S, double lmax, int m,
                            const double* const* coefs, const void* const* X, csc_dtype x_dt,
                            int64_t ldx, void* const* Y, csc_dtype y_dt, int64_t ldy, int w,
                            csc_dtype iter_dt, int variant, double* const* moments,
                            void* const* work, size_t work_bytes, hipStream_t s, bool timed);
csc_status run_gather_probe(const int32_t* rowptr, const int32_t* colidx, int64_t n,
                            const void* table, int row_bytes, uint32_t* out, hipStream_t s);
double filter_batch_bytes(const Graph* const* graphs, int S, int m, int w, csc_dtype iter_dt,
                          bool moments, csc_dtype y_dt);

// ------------------------------------------------------------------------------------
// reductions, RNG

csc_status launch_dot(const void* X, csc_dtype x_dt, int64_t ldx, const void* Y,
                      csc_dtype y_dt, int64_t ldy, int64_t n, int w, double* result,
                      void* work, size_t work_bytes, hipStream_t s);
size_t dot_workspace(int64_t n);

csc_status launch_randn(void* X, csc_dtype dt, int64_t n, int w, int64_t ldx, int64_t row0,
                        uint64_t seed, uint64_t stream_id, double sigma, hipStream_t s);
csc_status launch_uniforms(double* u, int count, uint64_t seed, uint64_t stream_id,
                           hipStream_t s);

// ------------------------------------------------------------------------------------
// k-means

size_t kmeans_workspace(int64_t n, int d, int k);
csc_status launch_kmeans_assign(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const float* C, int k, int32_t* labels, float* best_d2,
                                float* sums, int32_t* counts, void* work, size_t work_bytes,
                                hipStream_t s);
// the same assignment with its scratch in a static device array (no workspace, allocates
// nothing; k <= 240, d <= 256)
csc_status launch_kmeans_assign_static(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n,
                                       int d, const float* C, int k, int32_t* labels,
                                       float* best_d2, hipStream_t s);
size_t kmeans_static_scratch_bytes();
csc_status launch_kmeans_update(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const int32_t* labels, int k, float* C, int32_t* counts,
                                void* work, size_t work_bytes, hipStream_t s);
csc_status launch_kmeans_seed(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                              int k, const double* u, float* C, int32_t* idx, void* work,
                              size_t work_bytes, hipStream_t s);
csc_status run_kmeans(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                      int iters, int init, uint64_t seed, uint64_t stream_id, float* C,
                      int32_t* labels, double* objective, void* work, size_t work_bytes,
                      hipStream_t s);

// ------------------------------------------------------------------------------------
// host math

void cheb_coeffs(int m, double lmax, double lambda_c, csc_damping damp, double* a);
void bisect_moments(const double* mu, int m, double lmax, csc_damping damp, double sigma2,
                    int n_probe, double k, int n_cand, double lo, double hi, double* lambda_c,
                    double* count, double* trace);

// ------------------------------------------------------------------------------------
// timing

void timing_begin(hipStream_t s);
void timing_end(hipStream_t s, int64_t launches, double bytes);

}  // namespace csc

struct csc_graph_s {
  csc::Graph g;
};
