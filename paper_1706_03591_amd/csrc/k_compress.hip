// Compressive k-means (Sec. 2.2, Step 2): k-means on a random subset of the nodes, then the
// other assignments inferred by Tikhonov-regularised interpolation of the k cluster
// indicators.
//
//   1. weights w_i = ||theta_i||^2 (FP64, 8 lanes per row, fixed shuffle tree); prefix sums
//      by blocks of 1024 rows (fixed-order block sums, a sequential scan of the block sums);
//   2. n' draws: node i for uniform u when C_{i-1} <= u W < C_i (binary search over the
//      block offsets, then a scan inside the block);
//   3. the sampled rows gathered to FP32 and clustered with the library's k-means;
//   4. s_i = sum over the draws of node i of W / (n' w_i) (the diagonal of M^T P^-1 M) and
//      B[i, j] = the same sum over the draws of node i that landed in cluster j; duplicate
//      draws add identical values, so the atomic sums do not depend on their order;
//   5. (diag(s) + gamma L^r) X = B by conjugate gradients on all k columns together, with
//      the Jacobi-like preconditioner diag(s + gamma l^r), l the diagonal of L; each product
//      with L is one pass of the fused recurrence (degree-1 filter, lmax = 2: L = L~ + I);
//   6. labels = argmax_j X[i, j], ties to the lowest j.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kCT = 256;        // threads per block
constexpr int kScanRows = 1024;  // rows per prefix-sum block
constexpr int kNormLanes = 8;

template <typename T>
__device__ inline float ldf(const T* p, int64_t i);
template <>
__device__ inline float ldf<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ inline float ldf<uint16_t>(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }

template <typename T>
__global__ __launch_bounds__(kCT) void k_row_norm2(const T* F, int64_t ldf_, int64_t n, int d,
                                                   double* w) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  const int64_t r = t / kNormLanes;
  const int lane = static_cast<int>(t % kNormLanes);
  double acc = 0.0;
  if (r < n)
    for (int c = lane; c < d; c += kNormLanes) {
      const double v = ldf<T>(F, r * ldf_ + c);
      acc = fma(v, v, acc);
    }
#pragma unroll
  for (int off = 1; off < kNormLanes; off <<= 1) acc += __shfl_xor(acc, off, kNormLanes);
  if (r < n && lane == 0) w[r] = acc;
}

// Sum of rows [b * 1024, (b + 1) * 1024): four per thread in order, then a fixed tree.
__global__ __launch_bounds__(kCT) void k_block_sums(const double* w, int64_t n, double* bsum) {
  __shared__ double red[kCT];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kScanRows + threadIdx.x * 4;
  double s = 0.0;
  for (int i = 0; i < 4; ++i)
    if (r0 + i < n) s += w[r0 + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kCT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Exclusive scan of the block sums by one thread (a few thousand entries at most), and the
// total W in off[nb].
__global__ void k_scan_blocks(const double* bsum, int64_t nb, double* off) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double c = 0.0;
  for (int64_t b = 0; b < nb; ++b) {
    off[b] = c;
    c += bsum[b];
  }
  off[nb] = c;
}

__global__ __launch_bounds__(kCT) void k_draw(const double* u, int ns, const double* w, int64_t n,
                                              const double* off, int64_t nb, int32_t* idx) {
  const int s = blockIdx.x * kCT + threadIdx.x;
  if (s >= ns) return;
  const double target = u[s] * off[nb];
  // last block whose offset is <= target
  int64_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (off[mid] <= target) lo = mid; else hi = mid - 1;
  }
  const int64_t r0 = lo * kScanRows;
  const int64_t r1 = min(r0 + kScanRows, n);
  double c = off[lo];
  int64_t pick = -1, last = -1;
  for (int64_t i = r0; i < r1; ++i) {
    if (w[i] > 0.0) last = i;
    c += w[i];
    if (target < c) {
      pick = i;
      break;
    }
  }
  // rounding at the very end of a block: take its last row of positive weight
  idx[s] = static_cast<int32_t>(pick >= 0 ? pick : (last >= 0 ? last : r0));
}

template <typename T>
__global__ __launch_bounds__(kCT) void k_gather(const T* F, int64_t ldf_, const int32_t* idx, int ns,
                                                int d, float* Fs) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (t >= static_cast<int64_t>(ns) * d) return;
  const int64_t s = t / d;
  const int c = static_cast<int>(t % d);
  Fs[t] = ldf<T>(F, static_cast<int64_t>(idx[s]) * ldf_ + c);
}

__global__ __launch_bounds__(kCT) void k_zero_d(double* p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ __launch_bounds__(kCT) void k_rhs(const int32_t* idx, const int32_t* lab, int ns, int k,
                                             const double* w, const double* off, int64_t nb,
                                             double* sd, double* B) {
  const int s = blockIdx.x * kCT + threadIdx.x;
  if (s >= ns) return;
  const int64_t i = idx[s];
  const double v = off[nb] / (static_cast<double>(ns) * w[i]);
  atomicAdd(sd + i, v);
  const int j = lab[s];
  if (j >= 0 && j < k) atomicAdd(B + i * k + j, v);
}

// FP32 copies of s, the preconditioner s + gamma l^r, and B; X = 0, R = B, Z = B / pre, P = Z.
__global__ __launch_bounds__(kCT) void k_cg_init(const double* sd, const double* B, const float* diagL,
                                                 int64_t n, int k, float gamma, int r, float* s,
                                                 float* pre, float* X, float* R, float* Z, float* P) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (t >= n * k) return;
  const int64_t i = t / k;
  const float li = diagL ? diagL[i] : 1.f;
  float lr = 1.f;
  for (int q = 0; q < r; ++q) lr *= li;
  const float sv = static_cast<float>(sd[i]);
  const float pv = sv + gamma * lr;
  if (t % k == 0) {
    s[i] = sv;
    pre[i] = pv;
  }
  const float b = static_cast<float>(B[t]);
  X[t] = 0.f;
  R[t] = b;
  Z[t] = b / pv;
  P[t] = b / pv;
}

// Per-column <A_j, B_j> partials over row chunks of 256 rows (FP64, fixed order).
__global__ __launch_bounds__(kCT) void k_coldot_part(const float* A, const float* B, int64_t n, int k,
                                                     double* part) {
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kCT;
  const int64_t r1 = min(r0 + kCT, n);
  for (int j = threadIdx.x; j < k; j += kCT) {
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc = fma(static_cast<double>(A[r * k + j]), B[r * k + j], acc);
    part[static_cast<int64_t>(blockIdx.x) * k + j] = acc;
  }
}

__global__ __launch_bounds__(kCT) void k_coldot_final(const double* part, int64_t nb, int k, double* out) {
  for (int j = threadIdx.x; j < k; j += kCT) {
    double acc = 0.0;
    for (int64_t b = 0; b < nb; ++b) acc += part[b * k + j];
    out[j] = acc;
  }
}

// Q = s * P + gamma T
__global__ __launch_bounds__(kCT) void k_apply(const float* s, const float* P, const float* T,
                                               int64_t n, int k, float gamma, float* Q) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (t >= n * k) return;
  Q[t] = fmaf(s[t / k], P[t], gamma * T[t]);
}

// X += alpha_j P, R -= alpha_j Q, Z = R / pre
__global__ __launch_bounds__(kCT) void k_cg_update(const float* alpha, const float* pre, const float* P,
                                                   const float* Q, int64_t n, int k, float* X, float* R,
                                                   float* Z) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (t >= n * k) return;
  const float a = alpha[t % k];
  X[t] = fmaf(a, P[t], X[t]);
  const float rn = fmaf(-a, Q[t], R[t]);
  R[t] = rn;
  Z[t] = rn / pre[t / k];
}

// P = Z + beta_j P
__global__ __launch_bounds__(kCT) void k_cg_dir(const float* beta, const float* Z, int64_t n, int k,
                                                float* P) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (t >= n * k) return;
  P[t] = fmaf(beta[t % k], P[t], Z[t]);
}

__global__ __launch_bounds__(kCT) void k_argmax(const float* X, int64_t n, int k, int32_t* labels) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kCT + threadIdx.x;
  if (i >= n) return;
  int best = 0;
  float bv = X[i * k];
  for (int j = 1; j < k; ++j) {
    const float v = X[i * k + j];
    if (v > bv) {
      bv = v;
      best = j;
    }
  }
  labels[i] = best;
}

inline unsigned nblk(int64_t count) { return static_cast<unsigned>((count + kCT - 1) / kCT); }

struct CkLayout {
  size_t off_w, off_bsum, off_off, off_u, off_idx, off_fs, off_lab, off_c, off_sd, off_b, off_s,
      off_pre, off_x, off_r, off_z, off_p, off_q, off_t0, off_t1, off_part, off_dots, off_ab,
      off_km, off_fw, total;
  int64_t nb_scan, nb_dot;
};

CkLayout ck_layout(int64_t n, int d, int k, int ns) {
  CkLayout L{};
  L.nb_scan = (n + kScanRows - 1) / kScanRows;
  L.nb_dot = (n + kCT - 1) / kCT;
  const size_t nk = static_cast<size_t>(n) * k;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return o;
  };
  L.off_w = take(sizeof(double) * n);
  L.off_bsum = take(sizeof(double) * L.nb_scan);
  L.off_off = take(sizeof(double) * (L.nb_scan + 1));
  L.off_u = take(sizeof(double) * ns);
  L.off_idx = take(sizeof(int32_t) * ns);
  L.off_fs = take(sizeof(float) * static_cast<size_t>(ns) * d);
  L.off_lab = take(sizeof(int32_t) * ns);
  L.off_c = take(sizeof(float) * static_cast<size_t>(k) * d);
  L.off_sd = take(sizeof(double) * n);
  L.off_b = take(sizeof(double) * nk);
  L.off_s = take(sizeof(float) * n);
  L.off_pre = take(sizeof(float) * n);
  L.off_x = take(sizeof(float) * nk);
  L.off_r = take(sizeof(float) * nk);
  L.off_z = take(sizeof(float) * nk);
  L.off_p = take(sizeof(float) * nk);
  L.off_q = take(sizeof(float) * nk);
  L.off_t0 = take(sizeof(float) * nk);
  L.off_t1 = take(sizeof(float) * nk);
  L.off_part = take(sizeof(double) * static_cast<size_t>(L.nb_dot) * k);
  L.off_dots = take(sizeof(double) * 2 * k);
  L.off_ab = take(sizeof(float) * 2 * k);
  L.off_km = take(kmeans_workspace(ns, d, k));
  L.off_fw = take(filter_workspace(n, k, CSC_F32));
  L.total = off;
  return L;
}

}  // namespace

size_t compressive_workspace(int64_t n, int d, int k, int ns) { return ck_layout(n, d, k, ns).total; }

csc_status run_compressive(const Graph* g, const void* F, csc_dtype f_dt, int64_t ldf_, int d, int k,
                           int ns, int r, double gamma, int lloyd, int cg_iters, double cg_tol,
                           uint64_t seed, uint64_t sample_stream, uint64_t kmeans_stream,
                           int32_t* labels, int32_t* samples, int32_t* sample_labels, float* Xout,
                           int* iters_done, void* work, size_t work_bytes, hipStream_t st) {
  const int64_t n = g->n;
  if (!F || !labels) return fail(CSC_E_ARG, "null features or labels");
  if (f_dt != CSC_F32 && f_dt != CSC_BF16) return fail(CSC_E_DTYPE, "features must be F32 or BF16");
  if (d < 1 || ldf_ < d || k < 1 || k > 256 || ns < k || ns > n)
    return fail(CSC_E_ARG, "need 1 <= k <= 256, k <= n_sample <= n, ldf >= d >= 1");
  if (r < 1 || r > 8 || !(gamma > 0.0) || cg_iters < 1 || cg_iters > 100000 || !(cg_tol > 0.0))
    return fail(CSC_E_ARG, "need 1 <= r <= 8, gamma > 0, cg_iters >= 1, cg_tol > 0");
  const CkLayout L = ck_layout(n, d, k, ns);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "compressive workspace too small");
  char* base = static_cast<char*>(work);
  auto at = [&](size_t o) { return static_cast<void*>(base + o); };
  double* w = static_cast<double*>(at(L.off_w));
  double* bsum = static_cast<double*>(at(L.off_bsum));
  double* off = static_cast<double*>(at(L.off_off));
  double* u = static_cast<double*>(at(L.off_u));
  int32_t* idx = samples ? samples : static_cast<int32_t*>(at(L.off_idx));
  float* Fs = static_cast<float*>(at(L.off_fs));
  int32_t* lab = sample_labels ? sample_labels : static_cast<int32_t*>(at(L.off_lab));
  float* C = static_cast<float*>(at(L.off_c));
  double* sd = static_cast<double*>(at(L.off_sd));
  double* B = static_cast<double*>(at(L.off_b));
  float* s = static_cast<float*>(at(L.off_s));
  float* pre = static_cast<float*>(at(L.off_pre));
  float* X = Xout ? Xout : static_cast<float*>(at(L.off_x));
  float* R = static_cast<float*>(at(L.off_r));
  float* Z = static_cast<float*>(at(L.off_z));
  float* P = static_cast<float*>(at(L.off_p));
  float* Q = static_cast<float*>(at(L.off_q));
  float* T0 = static_cast<float*>(at(L.off_t0));
  float* T1 = static_cast<float*>(at(L.off_t1));
  double* part = static_cast<double*>(at(L.off_part));
  double* dots = static_cast<double*>(at(L.off_dots));
  float* ab = static_cast<float*>(at(L.off_ab));
  const int64_t nk = n * k;

  // 1-2: weights, prefix sums by blocks, draws
  if (f_dt == CSC_F32)
    hipLaunchKernelGGL(k_row_norm2<float>, dim3(nblk(n * kNormLanes)), dim3(kCT), 0, st,
                       static_cast<const float*>(F), ldf_, n, d, w);
  else
    hipLaunchKernelGGL(k_row_norm2<uint16_t>, dim3(nblk(n * kNormLanes)), dim3(kCT), 0, st,
                       static_cast<const uint16_t*>(F), ldf_, n, d, w);
  hipLaunchKernelGGL(k_block_sums, dim3(static_cast<unsigned>(L.nb_scan)), dim3(kCT), 0, st, w, n, bsum);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1), 0, st, bsum, L.nb_scan, off);
  CSC_TRY(launch_uniforms(u, ns, seed, sample_stream, st));
  hipLaunchKernelGGL(k_draw, dim3(nblk(ns)), dim3(kCT), 0, st, u, ns, w, n, off, L.nb_scan, idx);
  // 3: k-means on the sampled rows
  if (f_dt == CSC_F32)
    hipLaunchKernelGGL(k_gather<float>, dim3(nblk(static_cast<int64_t>(ns) * d)), dim3(kCT), 0, st,
                       static_cast<const float*>(F), ldf_, idx, ns, d, Fs);
  else
    hipLaunchKernelGGL(k_gather<uint16_t>, dim3(nblk(static_cast<int64_t>(ns) * d)), dim3(kCT), 0, st,
                       static_cast<const uint16_t*>(F), ldf_, idx, ns, d, Fs);
  CSC_HIP(hipGetLastError());
  CSC_TRY(run_kmeans(Fs, CSC_F32, d, ns, d, k, lloyd, 0, seed, kmeans_stream, C, lab, nullptr,
                     at(L.off_km), kmeans_workspace(ns, d, k), st));
  // 4: the diagonal of M^T P^-1 M and the right-hand sides
  hipLaunchKernelGGL(k_zero_d, dim3(nblk(n)), dim3(kCT), 0, st, sd, n);
  hipLaunchKernelGGL(k_zero_d, dim3(nblk(nk)), dim3(kCT), 0, st, B, nk);
  hipLaunchKernelGGL(k_rhs, dim3(nblk(ns)), dim3(kCT), 0, st, idx, lab, ns, k, w, off, L.nb_scan, sd, B);
  const float gam = static_cast<float>(gamma);
  hipLaunchKernelGGL(k_cg_init, dim3(nblk(nk)), dim3(kCT), 0, st, sd, B,
                     g->lap == CSC_LAP_COMBINATORIAL ? g->diag : nullptr, n, k, gam, r, s, pre, X, R, Z, P);
  CSC_HIP(hipGetLastError());

  // 5: preconditioned conjugate gradients, one independent system per column
  const double a1[2] = {1.0, 1.0};  // L x = (T_0 + T_1(L~)) x with lmax = 2
  auto coldots = [&](const float* A_, const float* B_, double* out) {
    hipLaunchKernelGGL(k_coldot_part, dim3(static_cast<unsigned>(L.nb_dot)), dim3(kCT), 0, st, A_, B_, n, k, part);
    hipLaunchKernelGGL(k_coldot_final, dim3(1), dim3(kCT), 0, st, part, L.nb_dot, k, out);
  };
  std::vector<double> h(2 * k), rz(k), bb(k);
  coldots(R, R, dots);
  coldots(R, Z, dots + k);
  CSC_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, st));
  CSC_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < k; ++j) {
    bb[j] = h[j];
    rz[j] = h[k + j];
  }
  std::vector<float> coef(k);
  int it = 0;
  for (; it < cg_iters; ++it) {
    // Q = (diag(s) + gamma L^r) P
    const float* src = P;
    for (int q = 0; q < r; ++q) {
      float* dst = (q & 1) ? T1 : T0;
      CSC_TRY(run_filter(g, 2.0, 1, a1, src, CSC_F32, k, dst, CSC_F32, k, k, CSC_F32, nullptr, 0,
                         at(L.off_fw), filter_workspace(n, k, CSC_F32), st));
      src = dst;
    }
    hipLaunchKernelGGL(k_apply, dim3(nblk(nk)), dim3(kCT), 0, st, s, P, src, n, k, gam, Q);
    coldots(P, Q, dots);
    CSC_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    CSC_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < k; ++j) coef[j] = (bb[j] > 0.0 && h[j] > 0.0) ? static_cast<float>(rz[j] / h[j]) : 0.f;
    CSC_HIP(hipMemcpyAsync(ab, coef.data(), sizeof(float) * k, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_cg_update, dim3(nblk(nk)), dim3(kCT), 0, st, ab, pre, P, Q, n, k, X, R, Z);
    coldots(R, R, dots);
    coldots(R, Z, dots + k);
    CSC_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, st));
    CSC_HIP(hipStreamSynchronize(st));
    double worst = 0.0;
    for (int j = 0; j < k; ++j)
      if (bb[j] > 0.0) worst = std::max(worst, std::sqrt(std::max(0.0, h[j]) / bb[j]));
    if (worst < cg_tol) {
      ++it;
      break;
    }
    for (int j = 0; j < k; ++j) {
      coef[j] = rz[j] > 0.0 ? static_cast<float>(h[k + j] / rz[j]) : 0.f;
      rz[j] = h[k + j];
    }
    CSC_HIP(hipMemcpyAsync(ab + k, coef.data(), sizeof(float) * k, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_cg_dir, dim3(nblk(nk)), dim3(kCT), 0, st, ab + k, Z, n, k, P);
  }
  // 6: assignments
  hipLaunchKernelGGL(k_argmax, dim3(nblk(n)), dim3(kCT), 0, st, X, n, k, labels);
  CSC_HIP(hipGetLastError());
  CSC_HIP(hipStreamSynchronize(st));
  if (iters_done) *iters_done = it;
  return CSC_OK;
}

}  // namespace csc
