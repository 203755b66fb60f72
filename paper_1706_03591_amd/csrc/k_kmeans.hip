// k-means on the rows of the spectral features (Sec. 2.1, eq. SC_cost): assignment,
// Lloyd update and k-means++ seeding, all with fixed-order reductions.
//
// Rows are served by groups of kG = 16 lanes; lane l of a group holds columns l, l + 16,
// l + 32, ... of its row, so a row load is coalesced and the centroid reads from LDS are
// broadcasts across the rows of a wave.  Distances to every centroid are ranked in FP32
// (direct form sum (f - mu)^2, so no cancellation), and the two best are re-scored in FP64
// so that the chosen label is the exact FP64 argmin of the two (ties to the lowest index).
#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kThreads = 256;
constexpr int kG = 16;             // lanes per row
constexpr int kMaxV = 16;          // columns per lane -> d <= 256
constexpr int kRowsPB = kThreads / kG;
constexpr int kLdsFloats = 12288;  // 48 KB of centroids per chunk

__device__ inline float ld_f(const void* F, int dt, int64_t i) {
  return dt == CSC_F32 ? static_cast<const float*>(F)[i]
                       : bf16_to_f32(static_cast<const uint16_t*>(F)[i]);
}

__device__ inline float grp_sum(float v) {
#pragma unroll
  for (int off = kG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kG);
  return v;
}
__device__ inline double grp_sum(double v) {
#pragma unroll
  for (int off = kG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kG);
  return v;
}

__device__ inline double block_sum(double v) {
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kThreads) void k_assign(const void* F, int f_dt, int64_t ldf,
                                                     int64_t n, int d, const float* C, int k,
                                                     int kc, int32_t* labels, float* best_d2,
                                                     double* obj_part) {
  __shared__ float s_c[kLdsFloats];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * kRowsPB + threadIdx.x / kG;
  const int lane = threadIdx.x % kG;
  const bool valid = row < n;
  const int nv = (d + kG - 1) / kG;
  float f[kMaxV];
#pragma unroll
  for (int i = 0; i < kMaxV; ++i) {
    const int col = lane + i * kG;
    f[i] = (valid && i < nv && col < d) ? ld_f(F, f_dt, row * ldf + col) : 0.f;
  }
  float b1 = INFINITY, b2 = INFINITY;
  int i1 = 0, i2 = -1;
  for (int c0 = 0; c0 < k; c0 += kc) {
    const int cn = min(kc, k - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < cn * d; t += kThreads) s_c[t] = C[static_cast<int64_t>(c0) * d + t];
    __syncthreads();
    for (int c = 0; c < cn; ++c) {
      const float* cc = s_c + c * d;
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < kMaxV; ++i) {
        const int col = lane + i * kG;
        if (i < nv && col < d) {
          const float t = f[i] - cc[col];
          s = fmaf(t, t, s);
        }
      }
      s = grp_sum(s);
      const int ci = c0 + c;
      if (s < b1) { b2 = b1; i2 = i1; b1 = s; i1 = ci; }
      else if (s < b2) { b2 = s; i2 = ci; }
    }
  }
  // FP64 re-score of the two best candidates
  double e1 = 0.0, e2 = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxV; ++i) {
    const int col = lane + i * kG;
    if (i < nv && col < d) {
      const double t1 = static_cast<double>(f[i]) - static_cast<double>(C[static_cast<int64_t>(i1) * d + col]);
      e1 += t1 * t1;
      if (i2 >= 0) {
        const double t2 = static_cast<double>(f[i]) - static_cast<double>(C[static_cast<int64_t>(i2) * d + col]);
        e2 += t2 * t2;
      }
    }
  }
  e1 = grp_sum(e1);
  e2 = grp_sum(e2);
  int lab = i1;
  double best = e1;
  if (i2 >= 0 && (e2 < e1 || (e2 == e1 && i2 < i1))) { lab = i2; best = e2; }
  if (valid && lane == 0) {
    labels[row] = lab;
    if (best_d2) best_d2[row] = static_cast<float>(best);
  }
  if (obj_part) {
    const double v = (valid && lane == 0) ? best : 0.0;
    const double s = block_sum(v);
    if (threadIdx.x == 0) obj_part[blockIdx.x] = s;
  }
}

// Per-block partial sums for the Lloyd update.  Block (b, y) owns rows [b * rpb, ...) and
// columns [64 y, 64 y + 64); `groups` copies of the k x 64 LDS accumulator let thread
// groups take interleaved rows; each thread owns one column, so every sum runs in a fixed
// order.  Counts come from column chunk 0.
__global__ void k_update_part(const void* F, int f_dt, int64_t ldf, int64_t n, int d,
                              const int32_t* labels, int k, int64_t rpb, int groups,
                              float* part, int32_t* cpart) {
  extern __shared__ float s_acc[];  // [groups][k][64] floats then [groups][k] ints
  int32_t* s_cnt = reinterpret_cast<int32_t*>(s_acc + static_cast<size_t>(groups) * k * 64);
  const int g = threadIdx.x / 64;
  const int cl = threadIdx.x % 64;
  const int col = blockIdx.y * 64 + cl;
  for (int t = threadIdx.x; t < groups * k * 64; t += blockDim.x) s_acc[t] = 0.f;
  for (int t = threadIdx.x; t < groups * k; t += blockDim.x) s_cnt[t] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rpb;
  const int64_t r1 = min(r0 + rpb, n);
  float* acc = s_acc + static_cast<size_t>(g) * k * 64;
  const bool colok = col < d;
  int64_t r = r0 + g;
  for (; r + 3 * groups < r1; r += 4 * groups) {
    const int la = labels[r], lb = labels[r + groups], lc = labels[r + 2 * groups],
              le = labels[r + 3 * groups];
    float va = 0.f, vb = 0.f, vc = 0.f, vd = 0.f;
    if (colok) {
      va = ld_f(F, f_dt, r * ldf + col);
      vb = ld_f(F, f_dt, (r + groups) * ldf + col);
      vc = ld_f(F, f_dt, (r + 2 * groups) * ldf + col);
      vd = ld_f(F, f_dt, (r + 3 * groups) * ldf + col);
    }
    acc[la * 64 + cl] += va;
    acc[lb * 64 + cl] += vb;
    acc[lc * 64 + cl] += vc;
    acc[le * 64 + cl] += vd;
    if (cl == 0 && blockIdx.y == 0) {
      s_cnt[g * k + la] += 1;
      s_cnt[g * k + lb] += 1;
      s_cnt[g * k + lc] += 1;
      s_cnt[g * k + le] += 1;
    }
  }
  for (; r < r1; r += groups) {
    const int la = labels[r];
    acc[la * 64 + cl] += colok ? ld_f(F, f_dt, r * ldf + col) : 0.f;
    if (cl == 0 && blockIdx.y == 0) s_cnt[g * k + la] += 1;
  }
  __syncthreads();
  if (colok) {
    for (int c = g; c < k; c += groups) {
      float s = 0.f;
      for (int q = 0; q < groups; ++q) s += s_acc[(static_cast<size_t>(q) * k + c) * 64 + cl];
      part[(static_cast<int64_t>(blockIdx.x) * k + c) * d + col] = s;
    }
  }
  if (blockIdx.y == 0) {
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
      int s = 0;
      for (int q = 0; q < groups; ++q) s += s_cnt[q * k + c];
      cpart[static_cast<int64_t>(blockIdx.x) * k + c] = s;
    }
  }
}

__global__ void k_update_final(const float* part, const int32_t* cpart, int64_t nblk, int k,
                               int d, float* C, int32_t* counts) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(k) * d) return;
  const int c = static_cast<int>(t / d);
  int64_t cnt = 0;
  for (int64_t b = 0; b < nblk; ++b) cnt += cpart[b * k + c];
  double s = 0.0;
  for (int64_t b = 0; b < nblk; ++b) s += static_cast<double>(part[b * k * d + t]);
  if (cnt > 0) C[t] = static_cast<float>(s / static_cast<double>(cnt));
  if (counts && (t % d) == 0) counts[c] = static_cast<int32_t>(cnt);
}

// ---------------- k-means++ ----------------

__global__ void k_pp_first(const void* F, int f_dt, int64_t ldf, int64_t n, int d,
                           const double* u, float* C, int32_t* idx, int32_t* sel) {
  int64_t i = static_cast<int64_t>(floor(u[0] * static_cast<double>(n)));
  if (i > n - 1) i = n - 1;
  if (i < 0) i = 0;
  if (threadIdx.x == 0) {
    sel[0] = static_cast<int32_t>(i);
    if (idx) idx[0] = static_cast<int32_t>(i);
  }
  for (int t = threadIdx.x; t < d; t += blockDim.x) C[t] = ld_f(F, f_dt, i * ldf + t);
}

// d2[i] = min(d2[i], ||f_i - C[j]||^2) in FP64 (first round: the distance itself); block
// sums of d2 in a fixed order.
__global__ __launch_bounds__(kThreads) void k_pp_dist(const void* F, int f_dt, int64_t ldf,
                                                      int64_t n, int d, const float* Cj, int first,
                                                      double* d2, double* bsum) {
  __shared__ double s_d[kRowsPB];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * kRowsPB + threadIdx.x / kG;
  const int lane = threadIdx.x % kG;
  double s = 0.0;
  if (row < n) {
    for (int col = lane; col < d; col += kG) {
      const double t = static_cast<double>(ld_f(F, f_dt, row * ldf + col)) - static_cast<double>(Cj[col]);
      s += t * t;
    }
  }
  s = grp_sum(s);
  if (lane == 0) {
    double v = 0.0;
    if (row < n) {
      v = first ? s : fmin(d2[row], s);
      d2[row] = v;
    }
    s_d[threadIdx.x / kG] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int i = 0; i < kRowsPB; ++i) b += s_d[i];
    bsum[blockIdx.x] = b;
  }
}

// Pick centre j: the first row whose running sum of d2 exceeds u[j] * total (running sum
// over the blocks' sums in block order, then over the rows of the crossing block in row
// order, the same order that formed each block sum).  One thread does the scan.
__global__ void k_pp_pick(const void* F, int f_dt, int64_t ldf, int64_t n, int d,
                          const double* d2, const double* bsum, int64_t nblk, const double* u,
                          int j, float* C, int32_t* idx, int32_t* sel) {
  __shared__ int64_t s_pick;
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int64_t b = 0; b < nblk; ++b) total += bsum[b];
    int64_t pick = sel[0];  // all distances zero: repeat the previous centre
    if (total > 0.0) {
      const double thr = u[j] * total;
      double run = 0.0;
      int64_t b = 0;
      while (b < nblk && run + bsum[b] <= thr) { run += bsum[b]; ++b; }
      if (b == nblk) { b = nblk - 1; run -= bsum[b]; }
      int64_t r = b * kRowsPB;
      const int64_t rend = min(r + kRowsPB, n);
      pick = rend - 1;
      for (; r < rend; ++r) {
        run += d2[r];
        if (run > thr) { pick = r; break; }
      }
    }
    s_pick = pick;
    sel[0] = static_cast<int32_t>(pick);
    if (idx) idx[j] = static_cast<int32_t>(pick);
  }
  __syncthreads();
  const int64_t pick = s_pick;
  for (int t = threadIdx.x; t < d; t += blockDim.x)
    C[static_cast<int64_t>(j) * d + t] = ld_f(F, f_dt, pick * ldf + t);
}

__global__ void k_sum_into(const double* part, int64_t nb, double* out) {
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kThreads) s += part[b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

struct KmLayout {
  int64_t nblk_upd, rpb, assign_blocks, pp_blocks;
  int groups;
  size_t off_u, off_d2, off_bsum, off_part, off_cpart, off_obj, off_objv, off_sel, total;
};

KmLayout km_layout(int64_t n, int d, int k) {
  KmLayout L{};
  L.assign_blocks = (n + kRowsPB - 1) / kRowsPB;
  L.pp_blocks = L.assign_blocks;
  const int64_t dch = (d + 63) / 64;
  (void)dch;
  int64_t nblk = std::max<int64_t>(1, std::min<int64_t>(2048, (n + 255) / 256));
  while (nblk > 64 && static_cast<double>(nblk) * k * d * 4.0 > 256.0 * 1024 * 1024) nblk /= 2;
  L.nblk_upd = nblk;
  L.rpb = (n + nblk - 1) / nblk;
  int groups = 4;
  while (groups > 1 && static_cast<size_t>(groups) * k * (64 * 4 + 4) > 60 * 1024) groups /= 2;
  L.groups = groups;
  size_t off = 0;
  L.off_u = off; off += align_up(static_cast<size_t>(k) * 8);
  L.off_d2 = off; off += align_up(static_cast<size_t>(n) * 8);
  L.off_bsum = off; off += align_up(static_cast<size_t>(L.pp_blocks) * 8);
  L.off_part = off; off += align_up(static_cast<size_t>(nblk) * k * d * 4);
  L.off_cpart = off; off += align_up(static_cast<size_t>(nblk) * k * 4);
  L.off_obj = off; off += align_up(static_cast<size_t>(L.assign_blocks) * 8);
  L.off_objv = off; off += align_up(static_cast<size_t>(1024 + 1) * 8);
  L.off_sel = off; off += 256;
  L.total = off;
  return L;
}

csc_status check_f(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                   bool need_k_le_n = false) {
  if (!F || n < 1 || d < 1 || ldf < d) return fail(CSC_E_ARG, "bad feature block");
  if (f_dt != CSC_F32 && f_dt != CSC_BF16) return fail(CSC_E_DTYPE, "features must be F32 or BF16");
  if (d > kG * kMaxV) return fail(CSC_E_ARG, "d must be <= 256");
  if (k < 1) return fail(CSC_E_ARG, "need k >= 1");
  if (need_k_le_n && k > n) return fail(CSC_E_ARG, "seeding needs k <= n");
  if (static_cast<size_t>(k) * (64 * 4 + 4) > 60 * 1024) return fail(CSC_E_ARG, "k too large (<= 235)");
  return CSC_OK;
}

}  // namespace

size_t kmeans_workspace(int64_t n, int d, int k) { return km_layout(n, d, k).total; }

csc_status launch_kmeans_assign(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const float* C, int k, int32_t* labels, float* best_d2,
                                double* obj_part, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  if (!C || !labels) return fail(CSC_E_ARG, "null centroids or labels");
  const int kc = std::max(1, std::min(k, kLdsFloats / d));
  const int64_t blocks = (n + kRowsPB - 1) / kRowsPB;
  hipLaunchKernelGGL(k_assign, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s, F,
                     int(f_dt), ldf, n, d, C, k, kc, labels, best_d2, obj_part);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status launch_kmeans_update(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const int32_t* labels, int k, float* C, int32_t* counts,
                                void* work, size_t work_bytes, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  const KmLayout L = km_layout(n, d, k);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "k-means workspace too small");
  char* base = static_cast<char*>(work);
  float* part = reinterpret_cast<float*>(base + L.off_part);
  int32_t* cpart = reinterpret_cast<int32_t*>(base + L.off_cpart);
  const size_t lds = static_cast<size_t>(L.groups) * k * 64 * 4 + static_cast<size_t>(L.groups) * k * 4;
  hipLaunchKernelGGL(k_update_part, dim3(static_cast<unsigned>(L.nblk_upd), (d + 63) / 64),
                     dim3(64 * L.groups), lds, s, F, int(f_dt), ldf, n, d, labels, k, L.rpb,
                     L.groups, part, cpart);
  const int64_t kd = static_cast<int64_t>(k) * d;
  hipLaunchKernelGGL(k_update_final, dim3(static_cast<unsigned>((kd + 255) / 256)), dim3(256), 0,
                     s, part, cpart, L.nblk_upd, k, d, C, counts);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status launch_kmeans_seed(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                              const double* u, float* C, int32_t* idx, void* work,
                              size_t work_bytes, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k, true));
  const KmLayout L = km_layout(n, d, k);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "k-means workspace too small");
  char* base = static_cast<char*>(work);
  double* d2 = reinterpret_cast<double*>(base + L.off_d2);
  double* bsum = reinterpret_cast<double*>(base + L.off_bsum);
  int32_t* sel = reinterpret_cast<int32_t*>(base + L.off_sel);
  hipLaunchKernelGGL(k_pp_first, dim3(1), dim3(256), 0, s, F, int(f_dt), ldf, n, d, u, C, idx, sel);
  for (int j = 1; j < k; ++j) {
    hipLaunchKernelGGL(k_pp_dist, dim3(static_cast<unsigned>(L.pp_blocks)), dim3(kThreads), 0, s,
                       F, int(f_dt), ldf, n, d, C + static_cast<int64_t>(j - 1) * d, j == 1 ? 1 : 0,
                       d2, bsum);
    hipLaunchKernelGGL(k_pp_pick, dim3(1), dim3(256), 0, s, F, int(f_dt), ldf, n, d, d2, bsum,
                       L.pp_blocks, u, j, C, idx, sel);
  }
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status run_kmeans(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                      int iters, int init, uint64_t seed, uint64_t stream_id, float* C,
                      int32_t* labels, double* objective, void* work, size_t work_bytes,
                      hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k, init == 0));
  if (iters < 0 || iters > 1024) return fail(CSC_E_ARG, "iters must be in [0, 1024]");
  const KmLayout L = km_layout(n, d, k);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "k-means workspace too small");
  char* base = static_cast<char*>(work);
  double* u = reinterpret_cast<double*>(base + L.off_u);
  double* obj = reinterpret_cast<double*>(base + L.off_obj);
  double* objv = reinterpret_cast<double*>(base + L.off_objv);
  if (init == 0) {
    CSC_TRY(launch_uniforms(u, k, seed, stream_id, s));
    CSC_TRY(launch_kmeans_seed(F, f_dt, ldf, n, d, k, u, C, nullptr, work, work_bytes, s));
  }
  for (int it = 0; it <= iters; ++it) {
    CSC_TRY(launch_kmeans_assign(F, f_dt, ldf, n, d, C, k, labels, nullptr,
                                 objective ? obj : nullptr, s));
    if (objective)
      hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(kThreads), 0, s, obj, L.assign_blocks, objv + it);
    if (it < iters)
      CSC_TRY(launch_kmeans_update(F, f_dt, ldf, n, d, labels, k, C, nullptr, work, work_bytes, s));
  }
  if (objective) {
    CSC_HIP(hipMemcpyAsync(objective, objv, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
  }
  return CSC_OK;
}

}  // namespace csc
