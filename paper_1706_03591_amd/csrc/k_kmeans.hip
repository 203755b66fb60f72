// k-means on the rows of the spectral features (Sec. 2.1, eq. SC_cost): assignment,
// Lloyd update and k-means++ seeding.
//
// Assignment: one lane per row.  Centroids are staged 32 at a time in LDS and read as
// broadcasts while each lane streams its row through registers 16 columns at a time, so
// the distances need no cross-lane reduction.  Distances are ranked in FP32 in the direct
// form sum (f - mu)^2 (no cancellation) and the two best candidates are re-scored in FP64,
// so the chosen label is the exact FP64 argmin of the two, ties going to the lowest index.
//
// Update: sums of the rows of each cluster in 64-bit fixed point (scale 2^S chosen from
// max |F| and n so that no sum can overflow), accumulated with integer atomics in LDS and
// then in global memory.  Integer addition is associative, so the sums do not depend on
// the order of the atomics and the update is bit-reproducible; the quantisation step
// 2^-S is far below FP32 resolution.
//
// k-means++: FP64 squared distances to the newest centre (one lane per row), block sums over
// contiguous row ranges, and a one-block pick of the first row whose running sum exceeds
// u_j * total.
#include <cmath>

#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kThreads = 256;

template <typename TF>
__device__ inline float to_f(TF v);
template <>
__device__ inline float to_f<float>(float v) { return v; }
template <>
__device__ inline float to_f<uint16_t>(uint16_t v) { return bf16_to_f32(v); }

__device__ inline double block_sum(double v) {
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < static_cast<int>(blockDim.x / 64); ++i) s += red[i];
  __syncthreads();
  return s;
}

// ---------------- assignment ----------------

constexpr int kKG = 32;   // centroids per staged group
constexpr int kCH = 16;   // columns per streamed chunk
constexpr int kRIT = 4;   // rows per thread per block

// kCH consecutive values of a row from column c0 (zeros past d).  Vector loads when the
// whole chunk is inside the row and rows are 16-byte aligned.
template <typename TF, bool VEC>
__device__ inline void load_chunk(const TF* rowp, int c0, int d, float* f) {
  if (VEC && c0 + kCH <= d) {
    const uint4* p = reinterpret_cast<const uint4*>(rowp + c0);
    if constexpr (sizeof(TF) == 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint4 u = p[q];
        f[4 * q] = __uint_as_float(u.x);
        f[4 * q + 1] = __uint_as_float(u.y);
        f[4 * q + 2] = __uint_as_float(u.z);
        f[4 * q + 3] = __uint_as_float(u.w);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint4 u = p[q];
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          f[8 * q + 2 * i] = __uint_as_float(w[i] << 16);
          f[8 * q + 2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < kCH; ++i) f[i] = (c0 + i < d) ? to_f<TF>(rowp[c0 + i]) : 0.f;
  }
}

// Each lane owns whole rows (kRIT of them per block pass).  The centroids come from a
// zero-padded copy Cp (kp x dp, kp a multiple of kKG): their addresses are uniform across
// the wave, so they are fetched with scalar loads and used as scalar operands of the FMAs
// while each lane streams its row through registers kCH columns at a time.  No LDS and no
// cross-lane reduction.  Top-2 in FP32 (increasing centroid index, strict <), then FP64
// re-score of the two.
template <typename TF, bool VEC>
__global__ __launch_bounds__(kThreads) void k_assign(const TF* F, int64_t ldf, int64_t n, int d,
                                                     int dp, const float* __restrict__ Cp, int k,
                                                     int32_t* labels, float* best_d2,
                                                     double* obj_part) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kRIT;
  double objsum = 0.0;
#pragma unroll 1
  for (int q = 0; q < kRIT; ++q) {
    const int64_t row = base + q * kThreads + threadIdx.x;
    const bool valid = row < n;
    const TF* rowp = F + (valid ? row : 0) * ldf;
    float b1 = INFINITY, b2 = INFINITY;
    int i1 = 0, i2 = -1;
#pragma unroll 1
    for (int g0 = 0; g0 < k; g0 += kKG) {
      float part[kKG];
#pragma unroll
      for (int cc = 0; cc < kKG; ++cc) part[cc] = 0.f;
#pragma unroll 1
      for (int c0 = 0; c0 < dp; c0 += kCH) {
        float f[kCH];
        if (valid) load_chunk<TF, VEC>(rowp, c0, d, f);
        else {
#pragma unroll
          for (int i = 0; i < kCH; ++i) f[i] = 0.f;
        }
#pragma unroll
        for (int cc = 0; cc < kKG; ++cc) {
          const float* cp = Cp + static_cast<int64_t>(g0 + cc) * dp + c0;
#pragma unroll
          for (int i = 0; i < kCH; ++i) {
            const float t = f[i] - cp[i];
            part[cc] = fmaf(t, t, part[cc]);
          }
        }
      }
      const int gn = min(kKG, k - g0);
#pragma unroll
      for (int cc = 0; cc < kKG; ++cc) {
        if (cc < gn) {
          const float sc = part[cc];
          if (sc < b1) { b2 = b1; i2 = i1; b1 = sc; i1 = g0 + cc; }
          else if (sc < b2) { b2 = sc; i2 = g0 + cc; }
        }
      }
    }
    if (!valid) continue;
    const float* c1 = Cp + static_cast<int64_t>(i1) * dp;
    const float* c2 = Cp + static_cast<int64_t>(i2 >= 0 ? i2 : i1) * dp;
    double e1 = 0.0, e2 = 0.0;
    for (int col = 0; col < d; ++col) {
      const double fv = static_cast<double>(to_f<TF>(rowp[col]));
      const double t1 = fv - static_cast<double>(c1[col]);
      const double t2 = fv - static_cast<double>(c2[col]);
      e1 += t1 * t1;
      e2 += t2 * t2;
    }
    int lab = i1;
    double best = e1;
    if (i2 >= 0 && (e2 < e1 || (e2 == e1 && i2 < i1))) { lab = i2; best = e2; }
    labels[row] = lab;
    if (best_d2) best_d2[row] = static_cast<float>(best);
    objsum += best;
  }
  if (obj_part) {
    const double s = block_sum(objsum);
    if (threadIdx.x == 0) obj_part[blockIdx.x] = s;
  }
}

// MFMA form of the assignment (when the centroids fit in LDS).  The cross term F C^T is a
// dense contraction, done with FP64 matrix cores (v_mfma_f64_16x16x4: A[i][k] from lane
// i + 16k, B[k][j] from lane j + 16k, output register r of lane l holds D[4r + l/16][l%16]).
// Each wave owns 16 rows at a time with the row values in registers (as doubles); the
// centroids are staged once per block in LDS (row stride DP + 1 to avoid bank conflicts)
// together with their FP64 squared norms.  Distances ||f||^2 - 2 f.c + ||c||^2 are formed in
// FP64 (cancellation error ~1e-16 ||f||^2, far below FP32 resolution), the two best are
// merged across lanes in (distance, index) order, and re-scored in the FP64 direct form so
// that exact ties still go to the lowest index.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int DP>
struct MfmaLds {
  static constexpr int kStride = DP + 1;
};

__device__ inline void top2_merge(double& b1, int& i1, double& b2, int& i2, double c1, int j1,
                                  double c2, int j2) {
  // merge two sorted (value, index) pairs lists of length two, keep the two smallest
  auto less = [](double va, int ia, double vb, int ib) { return va < vb || (va == vb && ia < ib); };
  double o1, o2;
  int p1, p2;
  if (less(b1, i1, c1, j1)) {
    o1 = b1; p1 = i1;
    if (less(b2, i2, c1, j1)) { o2 = b2; p2 = i2; } else { o2 = c1; p2 = j1; }
  } else {
    o1 = c1; p1 = j1;
    if (less(b1, i1, c2, j2)) { o2 = b1; p2 = i1; } else { o2 = c2; p2 = j2; }
  }
  b1 = o1; i1 = p1; b2 = o2; i2 = p2;
}

template <typename TF, int DP>
__global__ __launch_bounds__(256) void k_assign_mfma(const TF* F, int64_t ldf, int64_t n, int d,
                                                     const float* C, int k, int kp,
                                                     int32_t* labels, float* best_d2,
                                                     double* obj_part) {
  extern __shared__ float s_mem[];  // kp * (DP + 1) floats, then kp doubles
  constexpr int ST = MfmaLds<DP>::kStride;
  constexpr int NK = DP / 4;  // k-steps of the contraction
  float* s_c = s_mem;
  double* s_cn = reinterpret_cast<double*>(s_mem + ((kp * ST + 1) & ~1));
  for (int t = threadIdx.x; t < kp * ST; t += blockDim.x) {
    const int c = t / ST, col = t - c * ST;
    s_c[t] = (c < k && col < d) ? C[static_cast<int64_t>(c) * d + col] : 0.f;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kp; c += blockDim.x) {
    double q = 0.0;
    for (int col = 0; col < DP; ++col) {
      const double v = static_cast<double>(s_c[c * ST + col]);
      q += v * v;
    }
    s_cn[c] = q;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  double objsum = 0.0;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * waves + wave; tile < tiles;
       tile += static_cast<int64_t>(gridDim.x) * waves) {
    const int64_t row0 = tile * 16;
    // A operands: row row0 + li, columns lq + 4 i
    double a[NK];
    const int64_t arow = row0 + li;
    const bool avalid = arow < n;
    double fsq = 0.0;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const int col = lq + 4 * i;
      const double v = (avalid && col < d) ? static_cast<double>(to_f<TF>(F[arow * ldf + col])) : 0.0;
      a[i] = v;
      fsq += v * v;
    }
    fsq += __shfl_xor(fsq, 16, 64);
    fsq += __shfl_xor(fsq, 32, 64);  // ||f||^2 of row row0 + li, in every lane with that li
    double fn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) fn[r] = __shfl(fsq, 4 * r + lq, 64);  // rows 4 r + lq
    double b1[4], b2[4];
    int i1[4], i2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) { b1[r] = INFINITY; b2[r] = INFINITY; i1[r] = 0x7fffffff; i2[r] = 0x7fffffff; }
    for (int ct = 0; ct < kp / 16; ++ct) {
      mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
      const float* cb = s_c + (ct * 16 + li) * ST + lq;
#pragma unroll
      for (int i = 0; i < NK; ++i)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], static_cast<double>(cb[4 * i]), acc, 0, 0, 0);
      const int cent = ct * 16 + li;
      const double cn = s_cn[cent];
      if (cent < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double dist = fn[r] - 2.0 * acc[r] + cn;
          if (dist < b1[r]) { b2[r] = b1[r]; i2[r] = i1[r]; b1[r] = dist; i1[r] = cent; }
          else if (dist < b2[r]) { b2[r] = dist; i2[r] = cent; }
        }
      }
    }
    // merge the per-lane top-2 over the 16 lanes that share lq (one centroid column each)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const double c1 = __shfl_xor(b1[r], off, 64);
        const int j1 = __shfl_xor(i1[r], off, 64);
        const double c2 = __shfl_xor(b2[r], off, 64);
        const int j2 = __shfl_xor(i2[r], off, 64);
        top2_merge(b1[r], i1[r], b2[r], i2[r], c1, j1, c2, j2);
      }
    }
    // FP64 direct re-score of the two candidates when their expanded-form distances are
    // within a guard far above the expanded form's rounding (~1e-16 (||f||^2 + ||c||^2)), so
    // that exact ties still go to the lowest index; lanes li split the row's columns.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * r + lq;
      const bool valid = row < n;
      const int c1 = i1[r];
      const bool has2 = i2[r] < k;
      const int c2 = has2 ? i2[r] : c1;
      int lab = c1;
      double best = b1[r];
      const bool close = has2 && (b2[r] - b1[r]) <= 1e-10 * (fn[r] + fabs(b2[r]) + s_cn[c2]);
      if (close) {
        double e1 = 0.0, e2 = 0.0;
        for (int col = li; col < d; col += 16) {
          const double fv = valid ? static_cast<double>(to_f<TF>(F[row * ldf + col])) : 0.0;
          const double t1 = fv - static_cast<double>(s_c[c1 * ST + col]);
          const double t2 = fv - static_cast<double>(s_c[c2 * ST + col]);
          e1 += t1 * t1;
          e2 += t2 * t2;
        }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          e1 += __shfl_xor(e1, off, 16);
          e2 += __shfl_xor(e2, off, 16);
        }
        best = e1;
        if (e2 < e1 || (e2 == e1 && c2 < c1)) { lab = c2; best = e2; }
      } else {
        best = fmax(best, 0.0);
      }
      if (valid && li == 0) {
        labels[row] = lab;
        if (best_d2) best_d2[row] = static_cast<float>(best);
        objsum += best;
      }
    }
  }
  if (obj_part) {
    const double sm = block_sum(objsum);
    if (threadIdx.x == 0) obj_part[blockIdx.x] = sm;
  }
}

// Cp[c][col] = C[c][col] for c < k and col < d, zero elsewhere (kp x dp).
__global__ void k_pad_centroids(const float* C, int k, int d, int kp, int dp, float* Cp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kp * dp) return;
  const int c = t / dp, col = t - c * dp;
  Cp[t] = (c < k && col < d) ? C[static_cast<int64_t>(c) * d + col] : 0.f;
}

// ---------------- Lloyd update in fixed point ----------------

// Scale exponent S: every partial or total sum of n values below 2^e stays below 2^62.
__device__ inline int fixed_scale(float maxabs, int64_t n) {
  int e = 0;
  frexpf(maxabs, &e);  // maxabs < 2^e
  int ln = 0;
  while ((int64_t(1) << ln) < n) ++ln;
  int S = 62 - e - ln;
  return S < -60 ? -60 : (S > 120 ? 120 : S);
}

__global__ void k_upd_clear(unsigned long long* sums, int64_t kd, int32_t* cnt, int k,
                            uint32_t* maxabs) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < kd) sums[t] = 0ull;
  if (t < k) cnt[t] = 0;
  if (t == 0 && maxabs) maxabs[0] = 0u;
}

template <typename TF>
__global__ void k_maxabs(const TF* F, int64_t ldf, int64_t n, int d, uint32_t* out) {
  const int64_t total = n * d;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  float m = 0.f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t r = i / d;
    const int c = static_cast<int>(i - r * d);
    m = fmaxf(m, fabsf(to_f<TF>(F[r * ldf + c])));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Block (b, y): rows [b * rpb, ...), columns [y * cw, y * cw + cw).  LDS holds the k x cw
// fixed-point sums; thread groups take interleaved rows; integer atomics make the result
// independent of the order.
template <typename TF>
__global__ __launch_bounds__(kThreads) void k_upd_acc(const TF* F, int64_t ldf, int64_t n, int d,
                                                      const int32_t* labels, int k, int64_t rpb,
                                                      int cw, const uint32_t* maxabs,
                                                      unsigned long long* gsums, int32_t* gcnt) {
  extern __shared__ unsigned long long s_acc[];  // k * cw, then k ints
  int32_t* s_cnt = reinterpret_cast<int32_t*>(s_acc + static_cast<size_t>(k) * cw);
  for (int t = threadIdx.x; t < k * cw; t += kThreads) s_acc[t] = 0ull;
  for (int t = threadIdx.x; t < k; t += kThreads) s_cnt[t] = 0;
  __syncthreads();
  const int S = fixed_scale(__uint_as_float(maxabs[0]), n);
  const int groups = kThreads / cw;
  const int g = threadIdx.x / cw;
  const int cl = threadIdx.x % cw;
  const int col = blockIdx.y * cw + cl;
  const bool colok = col < d;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rpb;
  const int64_t r1 = min(r0 + rpb, n);
  const bool counter = cl == 0 && blockIdx.y == 0;
  int64_t r = r0 + g;
  for (; r + 3 * groups < r1; r += 4 * groups) {
    int lb[4];
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lb[q] = labels[r + q * groups];
      v[q] = colok ? to_f<TF>(F[(r + q * groups) * ldf + col]) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long fx = llrint(ldexp(static_cast<double>(v[q]), S));
      atomicAdd(&s_acc[lb[q] * cw + cl], static_cast<unsigned long long>(fx));
      if (counter) atomicAdd(&s_cnt[lb[q]], 1);
    }
  }
  for (; r < r1; r += groups) {
    const int lb = labels[r];
    const float v = colok ? to_f<TF>(F[r * ldf + col]) : 0.f;
    const long long fx = llrint(ldexp(static_cast<double>(v), S));
    atomicAdd(&s_acc[lb * cw + cl], static_cast<unsigned long long>(fx));
    if (counter) atomicAdd(&s_cnt[lb], 1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k * cw; t += kThreads) {
    const int c = t / cw, cc = t % cw;
    const int gc = blockIdx.y * cw + cc;
    if (gc < d && s_acc[t] != 0ull) atomicAdd(&gsums[static_cast<int64_t>(c) * d + gc], s_acc[t]);
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < k; t += kThreads)
      if (s_cnt[t]) atomicAdd(&gcnt[t], s_cnt[t]);
}

__global__ void k_upd_final(const unsigned long long* gsums, const int32_t* gcnt,
                            const uint32_t* maxabs, int64_t n, int k, int d, float* C,
                            int32_t* counts) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(k) * d) return;
  const int c = static_cast<int>(t / d);
  const int S = fixed_scale(__uint_as_float(maxabs[0]), n);
  const int32_t cnt = gcnt[c];
  if (cnt > 0) {
    const double sum = ldexp(static_cast<double>(static_cast<long long>(gsums[t])), -S);
    C[t] = static_cast<float>(sum / static_cast<double>(cnt));
  }
  if (counts && (t % d) == 0) counts[c] = cnt;
}

// ---------------- k-means++ ----------------

template <typename TF>
__global__ void k_pp_first(const TF* F, int64_t ldf, int64_t n, int d, const double* u, float* C,
                           int32_t* idx, int32_t* sel) {
  int64_t i = static_cast<int64_t>(floor(u[0] * static_cast<double>(n)));
  i = i > n - 1 ? n - 1 : (i < 0 ? 0 : i);
  if (threadIdx.x == 0) {
    sel[0] = static_cast<int32_t>(i);
    if (idx) idx[0] = static_cast<int32_t>(i);
  }
  for (int t = threadIdx.x; t < d; t += blockDim.x) C[t] = to_f<TF>(F[i * ldf + t]);
}

// d2[i] = min(d2[i], ||f_i - Cj||^2) in FP64 (first round: the distance itself); one lane
// per row, kRIT rows per thread, so block b covers the contiguous rows
// [b * kThreads * kRIT, ...); bsum[b] = their sum (fixed reduction order).
template <typename TF, bool VEC>
__global__ __launch_bounds__(kThreads) void k_pp_dist(const TF* F, int64_t ldf, int64_t n, int d,
                                                      int dp, const float* Cj, int first,
                                                      double* d2, double* bsum) {
  __shared__ float s_cj[256];
  for (int t = threadIdx.x; t < dp; t += kThreads) s_cj[t] = t < d ? Cj[t] : 0.f;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kRIT;
  double local = 0.0;
#pragma unroll 1
  for (int q = 0; q < kRIT; ++q) {
    const int64_t row = base + q * kThreads + threadIdx.x;
    if (row >= n) continue;
    const TF* rowp = F + row * ldf;
    double s = 0.0;
    for (int c0 = 0; c0 < dp; c0 += kCH) {
      float f[kCH];
      load_chunk<TF, VEC>(rowp, c0, d, f);
#pragma unroll
      for (int i = 0; i < kCH; ++i) {
        const double t = static_cast<double>(f[i]) - static_cast<double>(s_cj[c0 + i]);
        s += t * t;
      }
    }
    const double v = first ? s : fmin(d2[row], s);
    d2[row] = v;
    local += v;
  }
  const double tot = block_sum(local);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Inclusive prefix sums of v[0..1023] in LDS (Hillis-Steele, fixed order); 1024 threads.
__device__ inline void scan1024(double* v) {
  for (int off = 1; off < 1024; off <<= 1) {
    const double add = threadIdx.x >= static_cast<unsigned>(off) ? v[threadIdx.x - off] : 0.0;
    __syncthreads();
    v[threadIdx.x] += add;
    __syncthreads();
  }
}

// Pick centre j (1024 threads): prefix sums over chunks of block sums, the chunk and block
// where the running sum passes u_j * total, then a prefix scan of the rows of that block.
// Running sums are non-decreasing, so "first index above the threshold" is found by the one
// thread whose prefix crosses it.
template <typename TF>
__global__ __launch_bounds__(1024) void k_pp_pick(const TF* F, int64_t ldf, int64_t n, int d,
                                                  const double* d2, const double* bsum,
                                                  int64_t nblk, int64_t rows_per_blk,
                                                  const double* u, int j, float* C, int32_t* idx,
                                                  int32_t* sel) {
  __shared__ double s_v[1024];
  __shared__ int64_t s_at;
  __shared__ double s_base;
  const int t = threadIdx.x;
  const int64_t chunk = (nblk + 1023) / 1024;
  {
    double sum = 0.0;
    const int64_t b0 = static_cast<int64_t>(t) * chunk;
    for (int64_t b = b0; b < min(b0 + chunk, nblk); ++b) sum += bsum[b];
    s_v[t] = sum;
  }
  if (t == 0) s_at = -1;
  __syncthreads();
  scan1024(s_v);
  const double total = s_v[1023];
  const double thr = u[j] * total;
  if (total > 0.0) {
    const double prev = t > 0 ? s_v[t - 1] : 0.0;
    if (s_v[t] > thr && prev <= thr) { s_at = t; s_base = prev; }
  }
  __syncthreads();
  int64_t pick = sel[0];  // all distances zero: repeat the previous centre
  if (total > 0.0) {
    const int c = s_at >= 0 ? static_cast<int>(s_at) : 1023;
    __syncthreads();
    if (t == 0) {
      double run = s_at >= 0 ? s_base : (c > 0 ? s_v[c - 1] : 0.0);
      int64_t b = static_cast<int64_t>(c) * chunk;
      const int64_t bend = min(b + chunk, nblk);
      if (b >= nblk) b = nblk - 1;
      while (b < bend - 1 && run + bsum[b] <= thr) run += bsum[b++];
      s_at = b;
      s_base = run;
    }
    __syncthreads();
    const int64_t b = s_at;
    const double base = s_base;
    const int64_t r = b * rows_per_blk + t;
    __syncthreads();
    s_v[t] = (t < rows_per_blk && r < n) ? d2[r] : 0.0;
    if (t == 0) s_at = -1;
    __syncthreads();
    scan1024(s_v);
    const double prev = t > 0 ? s_v[t - 1] : 0.0;
    if (t < rows_per_blk && r < n && base + s_v[t] > thr && base + prev <= thr) s_at = r;
    __syncthreads();
    pick = s_at >= 0 ? s_at : min(b * rows_per_blk + rows_per_blk, n) - 1;
  }
  if (t == 0) {
    sel[0] = static_cast<int32_t>(pick);
    if (idx) idx[j] = static_cast<int32_t>(pick);
  }
  for (int q = t; q < d; q += blockDim.x)
    C[static_cast<int64_t>(j) * d + q] = to_f<TF>(F[pick * ldf + q]);
}

__global__ void k_sum_into(const double* part, int64_t nb, double* out) {
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kThreads) s += part[b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

// ---------------- dispatch ----------------

// Vector row loads need 16-byte aligned rows.
bool rows_aligned(const void* F, csc_dtype f_dt, int64_t ldf) {
  const size_t es = dtype_size(f_dt);
  return reinterpret_cast<uintptr_t>(F) % 16 == 0 && (static_cast<size_t>(ldf) * es) % 16 == 0;
}

int padded_d(int d) { return (d + kCH - 1) / kCH * kCH; }

int64_t assign_blocks(int64_t n) {
  const int64_t per = static_cast<int64_t>(kThreads) * kRIT;
  return std::max<int64_t>(1, (n + per - 1) / per);
}

struct KmLayout {
  size_t off_u, off_d2, off_bsum, off_sums, off_cnt, off_max, off_obj, off_objv, off_sel, off_cp,
      total;
};

int padded_k(int k) { return (k + kKG - 1) / kKG * kKG; }

KmLayout km_layout(int64_t n, int d, int k) {
  KmLayout L{};
  const int64_t blocks = assign_blocks(n);
  size_t off = 0;
  L.off_u = off; off += align_up(static_cast<size_t>(k) * 8);
  L.off_d2 = off; off += align_up(static_cast<size_t>(n) * 8);
  L.off_bsum = off; off += align_up(static_cast<size_t>(blocks) * 8);
  L.off_sums = off; off += align_up(static_cast<size_t>(k) * d * 8);
  L.off_cnt = off; off += align_up(static_cast<size_t>(k) * 4);
  L.off_max = off; off += 256;
  L.off_obj = off; off += align_up(static_cast<size_t>(std::max<int64_t>(blocks, 2048)) * 8);
  L.off_objv = off; off += align_up(static_cast<size_t>(1024 + 1) * 8);
  L.off_sel = off; off += 256;
  L.off_cp = off; off += align_up(static_cast<size_t>(padded_k(k)) * padded_d(d) * 4);
  L.total = off;
  return L;
}

csc_status check_f(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                   bool need_k_le_n = false) {
  if (!F || n < 1 || d < 1 || ldf < d) return fail(CSC_E_ARG, "bad feature block");
  if (f_dt != CSC_F32 && f_dt != CSC_BF16) return fail(CSC_E_DTYPE, "features must be F32 or BF16");
  if (d > 256) return fail(CSC_E_ARG, "d must be <= 256");
  if (k < 1) return fail(CSC_E_ARG, "need k >= 1");
  if (need_k_le_n && k > n) return fail(CSC_E_ARG, "seeding needs k <= n");
  if (static_cast<size_t>(k) * (32 * 8 + 4) > 62 * 1024) return fail(CSC_E_ARG, "k must be <= 240");
  return CSC_OK;
}

csc_status update_impl(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                       const int32_t* labels, int k, float* C, int32_t* counts, void* work,
                       bool max_ready, hipStream_t s) {
  const KmLayout L = km_layout(n, d, k);
  char* base = static_cast<char*>(work);
  auto* sums = reinterpret_cast<unsigned long long*>(base + L.off_sums);
  auto* cnt = reinterpret_cast<int32_t*>(base + L.off_cnt);
  auto* mx = reinterpret_cast<uint32_t*>(base + L.off_max);
  const int64_t kd = static_cast<int64_t>(k) * d;
  hipLaunchKernelGGL(k_upd_clear, dim3(static_cast<unsigned>((std::max<int64_t>(kd, k) + 255) / 256)),
                     dim3(256), 0, s, sums, kd, cnt, k, max_ready ? nullptr : mx);
  if (!max_ready) {
    const unsigned mblocks = static_cast<unsigned>(std::min<int64_t>(2048, (n * d + 255) / 256));
    if (f_dt == CSC_F32)
      hipLaunchKernelGGL(k_maxabs<float>, dim3(mblocks), dim3(256), 0, s, static_cast<const float*>(F),
                         ldf, n, d, mx);
    else
      hipLaunchKernelGGL(k_maxabs<uint16_t>, dim3(mblocks), dim3(256), 0, s,
                         static_cast<const uint16_t*>(F), ldf, n, d, mx);
  }
  const int cw = k <= 112 ? 64 : 32;
  const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>(2048, (n + 511) / 512));
  const int64_t rpb = (n + nblk - 1) / nblk;
  const size_t lds = static_cast<size_t>(k) * cw * 8 + static_cast<size_t>(k) * 4;
  const dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>((d + cw - 1) / cw));
  if (f_dt == CSC_F32)
    hipLaunchKernelGGL(k_upd_acc<float>, grid, dim3(kThreads), lds, s, static_cast<const float*>(F),
                       ldf, n, d, labels, k, rpb, cw, mx, sums, cnt);
  else
    hipLaunchKernelGGL(k_upd_acc<uint16_t>, grid, dim3(kThreads), lds, s,
                       static_cast<const uint16_t*>(F), ldf, n, d, labels, k, rpb, cw, mx, sums, cnt);
  hipLaunchKernelGGL(k_upd_final, dim3(static_cast<unsigned>((kd + 255) / 256)), dim3(256), 0, s,
                     sums, cnt, mx, n, k, d, C, counts);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace

size_t kmeans_workspace(int64_t n, int d, int k) { return km_layout(n, d, k).total; }

// LDS bytes of the MFMA assignment for (k, d), or 0 when it does not apply.
size_t mfma_lds_bytes(int k, int d, int* dp_out) {
  int dp = 16;
  while (dp < d) dp <<= 1;
  if (dp > 256) return 0;
  const int kp = (k + 15) / 16 * 16;
  const size_t bytes = static_cast<size_t>((kp * (dp + 1) + 1) & ~1) * 4 + static_cast<size_t>(kp) * 8;
  if (bytes > 48 * 1024) return 0;
  *dp_out = dp;
  return bytes;
}

int64_t mfma_blocks(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  return std::max<int64_t>(1, std::min<int64_t>(2048, (tiles + 3) / 4));
}

static csc_status assign_impl(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                              const float* C, int k, int32_t* labels, float* best_d2,
                              double* obj_part, float* Cp, hipStream_t s) {
  int dp2 = 0;
  const size_t mlds = mfma_lds_bytes(k, d, &dp2);
  if (mlds) {
    const unsigned blocks = static_cast<unsigned>(mfma_blocks(n));
    const int kp = (k + 15) / 16 * 16;
#define CSC_MF(TF, DPV)                                                                           \
  hipLaunchKernelGGL((k_assign_mfma<TF, DPV>), dim3(blocks), dim3(256), mlds, s,                  \
                     static_cast<const TF*>(F), ldf, n, d, C, k, kp, labels, best_d2, obj_part)
#define CSC_MF_DP(TF)                        \
  switch (dp2) {                             \
    case 16: CSC_MF(TF, 16); break;          \
    case 32: CSC_MF(TF, 32); break;          \
    case 64: CSC_MF(TF, 64); break;          \
    case 128: CSC_MF(TF, 128); break;        \
    default: CSC_MF(TF, 256); break;         \
  }
    if (f_dt == CSC_F32) { CSC_MF_DP(float) } else { CSC_MF_DP(uint16_t) }
#undef CSC_MF_DP
#undef CSC_MF
    CSC_HIP(hipGetLastError());
    return CSC_OK;
  }
  const bool vec = rows_aligned(F, f_dt, ldf);
  const unsigned blocks = static_cast<unsigned>(assign_blocks(n));
  const int dp = padded_d(d);
  const int kp = padded_k(k);
  hipLaunchKernelGGL(k_pad_centroids, dim3((kp * dp + 255) / 256), dim3(256), 0, s, C, k, d, kp, dp, Cp);
#define CSC_ASSIGN(TF, V)                                                                         \
  hipLaunchKernelGGL((k_assign<TF, V>), dim3(blocks), dim3(kThreads), 0, s,                       \
                     static_cast<const TF*>(F), ldf, n, d, dp, Cp, k, labels, best_d2, obj_part)
  if (f_dt == CSC_F32) {
    if (vec) CSC_ASSIGN(float, true); else CSC_ASSIGN(float, false);
  } else {
    if (vec) CSC_ASSIGN(uint16_t, true); else CSC_ASSIGN(uint16_t, false);
  }
#undef CSC_ASSIGN
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status launch_kmeans_assign(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const float* C, int k, int32_t* labels, float* best_d2,
                                double* obj_part, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  if (!C || !labels) return fail(CSC_E_ARG, "null centroids or labels");
  // the ABI call has no workspace: the padded centroids live in a small per-device buffer
  // owned by the library (grown on demand, kept until exit)
  static float* cp_buf = nullptr;
  static size_t cp_bytes = 0;
  const size_t need = static_cast<size_t>(padded_k(k)) * padded_d(d) * 4;
  if (need > cp_bytes) {
    if (cp_buf) (void)hipFree(cp_buf);
    cp_buf = nullptr;
    cp_bytes = 0;
    CSC_HIP(hipMalloc(&cp_buf, need));
    cp_bytes = need;
  }
  return assign_impl(F, f_dt, ldf, n, d, C, k, labels, best_d2, obj_part, cp_buf, s);
}

csc_status launch_kmeans_update(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                                const int32_t* labels, int k, float* C, int32_t* counts,
                                void* work, size_t work_bytes, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  const KmLayout L = km_layout(n, d, k);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "k-means workspace too small");
  return update_impl(F, f_dt, ldf, n, d, labels, k, C, counts, work, false, s);
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
  const bool vec = rows_aligned(F, f_dt, ldf);
  const int64_t rows_per_blk = static_cast<int64_t>(kThreads) * kRIT;
  const int64_t nblk = assign_blocks(n);
  const int dp = padded_d(d);
  const bool f32 = f_dt == CSC_F32;
  if (f32)
    hipLaunchKernelGGL(k_pp_first<float>, dim3(1), dim3(256), 0, s, static_cast<const float*>(F), ldf,
                       n, d, u, C, idx, sel);
  else
    hipLaunchKernelGGL(k_pp_first<uint16_t>, dim3(1), dim3(256), 0, s,
                       static_cast<const uint16_t*>(F), ldf, n, d, u, C, idx, sel);
#define CSC_PPD(TF, V)                                                                             \
  hipLaunchKernelGGL((k_pp_dist<TF, V>), dim3(static_cast<unsigned>(nblk)), dim3(kThreads), 0, s, \
                     static_cast<const TF*>(F), ldf, n, d, dp, Cj, first, d2, bsum)
  for (int j = 1; j < k; ++j) {
    const float* Cj = C + static_cast<int64_t>(j - 1) * d;
    const int first = j == 1 ? 1 : 0;
    if (f32) {
      if (vec) CSC_PPD(float, true); else CSC_PPD(float, false);
      hipLaunchKernelGGL(k_pp_pick<float>, dim3(1), dim3(1024), 0, s, static_cast<const float*>(F), ldf,
                         n, d, d2, bsum, nblk, rows_per_blk, u, j, C, idx, sel);
    } else {
      if (vec) CSC_PPD(uint16_t, true); else CSC_PPD(uint16_t, false);
      hipLaunchKernelGGL(k_pp_pick<uint16_t>, dim3(1), dim3(1024), 0, s,
                         static_cast<const uint16_t*>(F), ldf, n, d, d2, bsum, nblk, rows_per_blk, u,
                         j, C, idx, sel);
    }
  }
#undef CSC_PPD
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
  auto* mx = reinterpret_cast<uint32_t*>(base + L.off_max);
  if (init == 0) {
    CSC_TRY(launch_uniforms(u, k, seed, stream_id, s));
    CSC_TRY(launch_kmeans_seed(F, f_dt, ldf, n, d, k, u, C, nullptr, work, work_bytes, s));
  }
  // max |F| once: the features do not change during the Lloyd rounds
  hipLaunchKernelGGL(k_upd_clear, dim3(1), dim3(256), 0, s, static_cast<unsigned long long*>(nullptr),
                     int64_t(0), static_cast<int32_t*>(nullptr), 0, mx);
  {
    const unsigned mblocks = static_cast<unsigned>(std::min<int64_t>(2048, (n * d + 255) / 256));
    if (f_dt == CSC_F32)
      hipLaunchKernelGGL(k_maxabs<float>, dim3(mblocks), dim3(256), 0, s, static_cast<const float*>(F),
                         ldf, n, d, mx);
    else
      hipLaunchKernelGGL(k_maxabs<uint16_t>, dim3(mblocks), dim3(256), 0, s,
                         static_cast<const uint16_t*>(F), ldf, n, d, mx);
  }
  int dp2 = 0;
  const int64_t nparts = mfma_lds_bytes(k, d, &dp2) ? mfma_blocks(n) : assign_blocks(n);
  for (int it = 0; it <= iters; ++it) {
    CSC_TRY(assign_impl(F, f_dt, ldf, n, d, C, k, labels, nullptr, objective ? obj : nullptr,
                        reinterpret_cast<float*>(base + L.off_cp), s));
    if (objective)
      hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(kThreads), 0, s, obj, nparts, objv + it);
    if (it < iters) CSC_TRY(update_impl(F, f_dt, ldf, n, d, labels, k, C, nullptr, work, true, s));
  }
  if (objective) {
    CSC_HIP(hipMemcpyAsync(objective, objv, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
  }
  return CSC_OK;
}

}  // namespace csc
