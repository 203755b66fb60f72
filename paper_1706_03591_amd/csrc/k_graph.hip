// Operator build (Sec. 2.1), on the device, from the CSR weight matrix W: the normalized
// adjacency A = D^{-1/2} W D^{-1/2} (L = I - A), or W and the degrees (L = D - W), with
// optional validation of the CSR input (sorted rows, indices in range, no self-loops,
// positive weights, symmetry).  All accesses are bounds-checked, so an invalid input
// yields an error flag, never an out-of-range read.
#include <cstring>

#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kFlagRowptr = 1;
constexpr int kFlagIndex = 2;
constexpr int kFlagOrder = 4;
constexpr int kFlagSelf = 8;
constexpr int kFlagWeight = 16;
constexpr int kFlagSym = 32;

__global__ void k_check_rowptr(const int64_t* rowptr, int64_t n, int64_t nnz, int32_t* flags) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r > n) return;
  int64_t v = rowptr[r];
  bool bad = v < 0 || v > nnz;
  if (r == 0 && v != 0) bad = true;
  if (r == n && v != nnz) bad = true;
  if (r < n && rowptr[r + 1] < v) bad = true;
  if (bad) atomicOr(flags, kFlagRowptr);
}

// One thread per row; assumes k_check_rowptr passed (checked on the host in between).
__global__ void k_check_rows(const int64_t* rowptr, const int32_t* colidx, const double* w,
                             int64_t n, int32_t* flags) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t s = rowptr[r], e = rowptr[r + 1];
  int bad = 0;
  int64_t prev = -1;
  for (int64_t i = s; i < e; ++i) {
    int64_t c = colidx[i];
    double wi = w[i];
    if (c < 0 || c >= n) { bad |= kFlagIndex; continue; }
    if (c <= prev) bad |= kFlagOrder;
    prev = c;
    if (c == r) bad |= kFlagSelf;
    if (!(wi > 0.0) || !(wi < INFINITY)) bad |= kFlagWeight;
    // symmetric partner (c, r) by binary search in row c
    int64_t lo = rowptr[c], hi = rowptr[c + 1] - 1;
    bool found = false;
    while (lo <= hi) {
      int64_t mid = (lo + hi) >> 1;
      int64_t cm = colidx[mid];
      if (cm == r) { found = (w[mid] == wi); break; }
      if (cm < r) lo = mid + 1; else hi = mid - 1;
    }
    if (!found) bad |= kFlagSym;
  }
  if (bad) atomicOr(flags, bad);
}

__global__ void k_rowptr32(const int64_t* rowptr, int32_t* out, int64_t n) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r <= n) out[r] = static_cast<int32_t>(rowptr[r]);
}

// kLPR lanes per row: each lane sums a strided subset of the row's weights, then a fixed
// shuffle tree combines them, so the degree does not depend on scheduling.
constexpr int kLPR = 8;

__global__ void k_degrees(const int64_t* rowptr, const double* w, int64_t n, double* dinv,
                          double* deg_out, float* diag_out, int32_t* isolated) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = t / kLPR;
  const int lane = static_cast<int>(t % kLPR);
  double deg = 0.0;
  int64_t rs = 0, re = 0;
  if (r < n) {
    rs = rowptr[r];
    re = rowptr[r + 1];
    for (int64_t i = rs + lane; i < re; i += kLPR) deg += w[i];
  }
#pragma unroll
  for (int off = 1; off < kLPR; off <<= 1) deg += __shfl_xor(deg, off, kLPR);
  if (r < n && lane == 0) {
    dinv[r] = deg > 0.0 ? 1.0 / sqrt(deg) : 0.0;
    if (deg_out) deg_out[r] = deg;
    if (diag_out) diag_out[r] = static_cast<float>(deg);
    if (re == rs) atomicAdd(isolated, 1);
  }
}

// Anderson-Morley bound max over stored entries (r, c) of d_r + d_c.  The sums are
// non-negative doubles, whose bit patterns order like the values, so an integer atomic
// maximum on the bits finds the largest.
__global__ void k_am_bound(const int64_t* rowptr, const int32_t* colidx, const double* deg,
                           int64_t n, unsigned long long* out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = t / kLPR;
  const int lane = static_cast<int>(t % kLPR);
  double best = 0.0;
  if (r < n) {
    const double dr = deg[r];
    for (int64_t i = rowptr[r] + lane; i < rowptr[r + 1]; i += kLPR)
      best = fmax(best, dr + deg[colidx[i]]);
  }
#pragma unroll
  for (int off = 1; off < kLPR; off <<= 1) best = fmax(best, __shfl_xor(best, off, kLPR));
  if (r < n && lane == 0 && best > 0.0) atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(best)));
}

template <typename TV>
__device__ inline TV to_val(double x);
template <>
__device__ inline float to_val<float>(double x) { return static_cast<float>(x); }
template <>
__device__ inline uint16_t to_val<uint16_t>(double x) {
  return f32_to_bf16(static_cast<float>(x));
}

// Stored values: w_rc d_r^{-1/2} d_c^{-1/2} (normalized), or w_rc itself (dinv null).
template <typename TV>
__global__ void k_values(const int64_t* rowptr, const int32_t* colidx, const double* w,
                         const double* dinv, int64_t n, int32_t* colidx_out, TV* vals) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = t / kLPR;
  const int lane = static_cast<int>(t % kLPR);
  if (r >= n) return;
  const double dr = dinv ? dinv[r] : 1.0;
  for (int64_t i = rowptr[r] + lane; i < rowptr[r + 1]; i += kLPR) {
    const int32_t c = colidx[i];
    colidx_out[i] = c;
    vals[i] = to_val<TV>(dinv ? w[i] * dr * dinv[c] : w[i]);
  }
}

// mirror[e] = index of entry (c, r) for entry e = (r, c); one thread per row.
__global__ void k_mirror(const int32_t* rowptr, const int32_t* colidx, int64_t n,
                         int32_t* mirror) {
  int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int32_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
    int32_t c = colidx[i];
    int32_t lo = rowptr[c], hi = rowptr[c + 1] - 1, pos = -1;
    while (lo <= hi) {
      int32_t mid = (lo + hi) >> 1;
      int32_t cm = colidx[mid];
      if (cm == r) { pos = mid; break; }
      if (cm < r) lo = mid + 1; else hi = mid - 1;
    }
    mirror[i] = pos;
  }
}

__device__ inline float load_val(const void* v, int dt, int64_t i) {
  if (dt == CSC_F32) return static_cast<const float*>(v)[i];
  return bf16_to_f32(static_cast<const uint16_t*>(v)[i]);
}

// Chain of the adjoint from A to the edge weights (normalized Laplacian, Sec. 2.1:
// A = D^{-1/2} W D^{-1/2}, d = W 1; s = D^{-1/2}).  With G_e = dl/dA_e per stored entry:
//   q_r = sum over the entries e of row r of G_e A_e + G_m(e) A_m(e)   (m(e) the mirror)
//   g_e = G_e s_r s_c - q_r s_r^2 / 2                                  (W_rc as a parameter)
//   dW_e = g_e + g_m(e)                    (the undirected weight, stored twice)
// FP64 throughout, each sum in entry order; one thread per row.
__global__ void k_wgrad_q(const int32_t* rowptr, const int32_t* mirror, const void* vals, int dt,
                          const float* dA, int64_t n, double* q) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int32_t me = mirror[e];
    acc += static_cast<double>(dA[e]) * static_cast<double>(load_val(vals, dt, e));
    acc += static_cast<double>(dA[me]) * static_cast<double>(load_val(vals, dt, me));
  }
  q[r] = acc;
}

__global__ void k_wgrad(const int32_t* rowptr, const int32_t* colidx, const int32_t* mirror,
                        const double* dinv, const float* dA, const double* q, int64_t n,
                        double* dW) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double sr = dinv[r];
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int32_t c = colidx[e];
    const double sc = dinv[c];
    const double g = static_cast<double>(dA[e]) * sr * sc - 0.5 * q[r] * sr * sr;
    const double gm = static_cast<double>(dA[mirror[e]]) * sc * sr - 0.5 * q[c] * sc * sc;
    dW[e] = g + gm;
  }
}

// Edge distance (Sec. 4): per row, the two sorted column lists are merged and the squared
// differences of the stored off-diagonal values summed in FP64 (an entry present in one
// graph only counts with the other's value 0); for L = D - W the squared difference of the
// degrees is added.  One thread per row; fixed-order block tree, one partial per block.
constexpr int kDistThreads = 256;

struct DistSide {
  const int32_t* rowptr;
  const int32_t* colidx;
  const void* vals;
  int dt;
  const double* deg;
};

__global__ __launch_bounds__(kDistThreads) void k_edge_dist(DistSide a, DistSide b, int64_t n,
                                                            double* part) {
  __shared__ double red[kDistThreads];
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kDistThreads + threadIdx.x;
  double sum = 0.0;
  if (r < n) {
    int32_t i = a.rowptr[r];
    const int32_t ie = a.rowptr[r + 1];
    int32_t j = b.rowptr[r];
    const int32_t je = b.rowptr[r + 1];
    while (i < ie || j < je) {
      const int32_t ca = i < ie ? a.colidx[i] : INT32_MAX;
      const int32_t cb = j < je ? b.colidx[j] : INT32_MAX;
      double dv;
      if (ca == cb) {
        dv = static_cast<double>(load_val(b.vals, b.dt, j)) - load_val(a.vals, a.dt, i);
        ++i;
        ++j;
      } else if (ca < cb) {
        dv = load_val(a.vals, a.dt, i);
        ++i;
      } else {
        dv = load_val(b.vals, b.dt, j);
        ++j;
      }
      sum = fma(dv, dv, sum);
    }
    if (a.deg) {
      const double dd = b.deg[r] - a.deg[r];
      sum = fma(dd, dd, sum);
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int h = kDistThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kDistThreads) void k_sum_parts(const double* part, int64_t np,
                                                            double* out) {
  __shared__ double red[kDistThreads];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += kDistThreads) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kDistThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

inline unsigned blocks_for(int64_t count, int threads = 256) {
  return static_cast<unsigned>((count + threads - 1) / threads);
}

std::string flag_text(int f) {
  std::string s;
  if (f & kFlagRowptr) s += " row pointers not monotone or out of [0, nnz];";
  if (f & kFlagIndex) s += " column index out of range;";
  if (f & kFlagOrder) s += " columns not strictly increasing within a row;";
  if (f & kFlagSelf) s += " self-loop;";
  if (f & kFlagWeight) s += " weight not positive and finite;";
  if (f & kFlagSym) s += " W not symmetric;";
  return s;
}

}  // namespace

csc_status graph_build(Graph* g, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                       const double* w, int validate, hipStream_t s) {
  const int64_t n = g->n;
  CSC_HIP(hipMemsetAsync(g->flags, 0, 4 * sizeof(int32_t), s));
  if (validate) {
    hipLaunchKernelGGL(k_check_rowptr, dim3(blocks_for(n + 1)), dim3(256), 0, s, rowptr, n,
                       nnz, g->flags);
    CSC_HIP(hipGetLastError());
    int32_t f = 0;
    CSC_HIP(hipMemcpyAsync(&f, g->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (f) return fail(CSC_E_GRAPH, "invalid CSR graph:" + flag_text(f));
    if (nnz > 0) {
      hipLaunchKernelGGL(k_check_rows, dim3(blocks_for(n)), dim3(256), 0, s, rowptr, colidx, w,
                         n, g->flags);
      CSC_HIP(hipGetLastError());
      CSC_HIP(hipMemcpyAsync(&f, g->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      CSC_HIP(hipStreamSynchronize(s));
      if (f) return fail(CSC_E_GRAPH, "invalid CSR graph:" + flag_text(f));
    }
  }
  g->nnz = nnz;
  hipLaunchKernelGGL(k_rowptr32, dim3(blocks_for(n + 1)), dim3(256), 0, s, rowptr, g->rowptr, n);
  const bool comb = g->lap == CSC_LAP_COMBINATORIAL;
  hipLaunchKernelGGL(k_degrees, dim3(blocks_for(n * kLPR)), dim3(256), 0, s, rowptr, w, n, g->dinv,
                     comb ? g->deg : nullptr, comb ? g->diag : nullptr, g->flags + 1);
  const double* scale = comb ? nullptr : g->dinv;
  if (g->val_dt == CSC_F32)
    hipLaunchKernelGGL(k_values<float>, dim3(blocks_for(n * kLPR)), dim3(256), 0, s, rowptr, colidx,
                       w, scale, n, g->colidx, static_cast<float*>(g->vals));
  else
    hipLaunchKernelGGL(k_values<uint16_t>, dim3(blocks_for(n * kLPR)), dim3(256), 0, s, rowptr,
                       colidx, w, scale, n, g->colidx, static_cast<uint16_t*>(g->vals));
  g->mirror_valid = false;
  CSC_HIP(hipGetLastError());
  if (comb) {
    // flags[2..3] hold the bound's bits (zeroed with the flags above)
    auto* bits = reinterpret_cast<unsigned long long*>(g->flags + 2);
    hipLaunchKernelGGL(k_am_bound, dim3(blocks_for(n * kLPR)), dim3(256), 0, s, rowptr, colidx,
                       g->deg, n, bits);
    CSC_HIP(hipGetLastError());
    unsigned long long b = 0;
    CSC_HIP(hipMemcpyAsync(&b, bits, sizeof(b), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    double v = 0.0;
    std::memcpy(&v, &b, sizeof(v));
    g->lmax_bound = v > 0.0 ? v : 1.0;
  } else {
    g->lmax_bound = 2.0;
  }
  return CSC_OK;
}

size_t distance_workspace(int64_t n) {
  return static_cast<size_t>((n + kDistThreads - 1) / kDistThreads) * sizeof(double);
}

csc_status graph_distance2(const Graph* a, const Graph* b, double* out, void* work,
                           size_t work_bytes, hipStream_t s) {
  if (a->n != b->n) return fail(CSC_E_ARG, "graphs of different sizes");
  if (a->lap != b->lap) return fail(CSC_E_ARG, "graphs of different Laplacian kinds");
  if (!out || !work || work_bytes < distance_workspace(a->n))
    return fail(CSC_E_ARG, "distance workspace too small");
  const bool comb = a->lap == CSC_LAP_COMBINATORIAL;
  const DistSide da{a->rowptr, a->colidx, a->vals, int(a->val_dt), comb ? a->deg : nullptr};
  const DistSide db{b->rowptr, b->colidx, b->vals, int(b->val_dt), comb ? b->deg : nullptr};
  const int64_t nb = (a->n + kDistThreads - 1) / kDistThreads;
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL(k_edge_dist, dim3(static_cast<unsigned>(nb)), dim3(kDistThreads), 0, s, da, db,
                     a->n, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kDistThreads), 0, s, part, nb, out);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// The mirror index is needed only by the adjoint and by csc_graph_arrays; it is built on
// first use after each (re)build.
csc_status graph_weight_grad(Graph* g, const float* dA, double* dW, double* q, hipStream_t s) {
  if (g->lap != CSC_LAP_NORMALIZED) return fail(CSC_E_ARG, "the weight chain is for the normalized Laplacian");
  if (g->n == 0) return CSC_OK;
  CSC_TRY(graph_ensure_mirror(g, s));
  hipLaunchKernelGGL(k_wgrad_q, dim3(blocks_for(g->n)), dim3(256), 0, s, g->rowptr, g->mirror,
                     static_cast<const void*>(g->vals), int(g->val_dt), dA, g->n, q);
  hipLaunchKernelGGL(k_wgrad, dim3(blocks_for(g->n)), dim3(256), 0, s, g->rowptr, g->colidx,
                     g->mirror, g->dinv, dA, static_cast<const double*>(q), g->n, dW);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status graph_ensure_mirror(Graph* g, hipStream_t s) {
  if (g->mirror_valid) return CSC_OK;
  hipLaunchKernelGGL(k_mirror, dim3(blocks_for(g->n)), dim3(256), 0, s, g->rowptr, g->colidx, g->n,
                     g->mirror);
  CSC_HIP(hipGetLastError());
  g->mirror_valid = true;
  return CSC_OK;
}

}  // namespace csc
