// k-means on the rows of the spectral features (Sec. 2.1, eq. SC_cost): assignment,
// Lloyd update and k-means++ seeding.
//
// Assignment (d <= 256, aligned rows): the cross term on the BF16 matrix cores in exact
// split precision with a certified error bound; a row whose certified candidates are two
// is re-scored in FP64 against both, a row with more against every centroid.  Fallback
// (wider or unaligned rows): one lane per row, scalar-broadcast centroids, FP32 direct-form
// ranking and FP64 re-score of the best two.
//
// Update: sums of the rows of each cluster in 64-bit fixed point (scale 2^S chosen from
// max |F| and n so that no sum can overflow).  The rows are ordered by label (counting
// sort), summed in chunks of one label each, and the chunk sums added per label.  Integer
// addition is associative, so the sums depend neither on the order of the rows within a
// label nor on the chunking, and the update is bit-reproducible; the quantisation step
// 2^-S is far below FP32 resolution.
//
// k-means++: FP64 squared distances to the newest centre (sixteen lanes per row, rows the
// triangle inequality rules out are not read), block sums over contiguous row ranges, and a
// one-block pick of the first row whose running sum exceeds u_j * total.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "csc_internal.h"

namespace csc {

size_t assign_scratch_bytes(int k, int d);

namespace {

constexpr int kThreads = 256;

template <typename TF>
__device__ inline float to_f(TF v);
template <>
__device__ inline float to_f<float>(float v) { return v; }
template <>
__device__ inline float to_f<uint16_t>(uint16_t v) { return bf16_to_f32(v); }

__device__ inline double block_sum(double v) {
  __shared__ double red[16];  // blocks of up to 1024 threads
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
constexpr int kGroup = 2; // 32-column MFMA steps per fresh FP32 accumulator in the assignment
constexpr int kCParts = 2; // BF16 parts of a centroid value on the matrix cores (hi, mid)
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

// MFMA form of the assignment (d <= 256).  The cross term F C^T is a dense contraction and
// runs on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) in split precision: each FP32
// centroid value is rounded to two BF16 parts (hi, mid); what they leave out, r_c (at most
// 2^-16 of each value), moves a dot product by at most ||f|| ||r_c||, with ||r_c|| computed
// exactly per centroid.  Each FP32 feature is split into three BF16 parts (BF16 features are
// their own single part), so every partial product is exact in FP32.  Each pair of 32-column steps of the dominant hi x hi product
// goes into a fresh FP32 accumulator (at most 64 u of rounding, u = 2^-24, relative to the
// sum of its absolute products), the at most four pairs are summed in FP32 (at most 3 u
// more), and the small cross products (weights 2^-8 and below) of each pair are summed in
// FP32 into a second accumulator (5 u covers them and the dropped row-part products).  A dot
// product is then within E ||f|| ||c|| + ||f|| ||r_c|| of f.c with E = 72 2^-24.  The score
// s_c = ||c||^2 - 2 f.c and its ends are formed in FP32, so the exact score lies in
// [s_c - e_c, s_c + e_c] with e_c = (2 E + 16 u) ||f|| ||c|| + 2 ||f|| ||r_c|| + 8 u ||c||^2 +
// 2^-110: the u
// terms bound the FP32 rounding of ||c||^2, of the two sums, of the score and of its ends
// (each at most u times ||c||^2 + 2 ||f|| ||c||), and the absolute term covers products that
// underflow, so such rows are re-scored rather than misassigned.  The argmin is then
// among the centroids whose lower end is below the smallest upper end.  Each lane keeps its
// three smallest lower ends and the smallest upper end; after the merge across lanes a row
// with one such candidate is certified, a row with two is re-scored against both in the
// FP64 direct form, and any other row against every centroid.  The direct form is the
// definition of the assignment, and ties go to the lowest index.
//
// Work layout: a wave owns 16 rows at a time (A operand: lane l holds row l % 16, eight
// consecutive columns per 32-column step starting at 8 (l / 16)); the centroid parts are
// staged in LDS in chunks of up to kc_max centroids, 16-byte padded rows so that the sixteen
// centroid rows read by one MFMA start in different banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// row of the MFMA output held in register r of a lane in row group lq
__device__ constexpr int mf_drow(int r, int lq) { return 4 * lq + r; }

__host__ __device__ inline void split3(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
  h = f32_to_bf16(x);
  float rem = x - bf16_to_f32(h);
  m = f32_to_bf16(rem);
  rem = rem - bf16_to_f32(m);
  l = f32_to_bf16(rem);
}

// parts[(p * kp + c) * DP + col], p = 0 hi, 1 mid (the lo part is dropped: its value, at most
// 2^-16 of the centroid value, is carried by the score's error bound); zero for c >= k or
// col >= d.
__global__ void k_prep_centroids(const float* C, int k, int d, int kp, int DP, uint16_t* parts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kp * DP) return;
  const int c = t / DP, col = t - c * DP;
  const float x = (c < k && col < d) ? C[static_cast<int64_t>(c) * d + col] : 0.f;
  uint16_t h, m, l;
  split3(x, h, m, l);
  parts[t] = h;
  parts[static_cast<int64_t>(kp) * DP + t] = m;
}

// cn[c] = ||C_c||^2 in FP64 for c < k, +inf for the padding up to kp, and cn[kp + c] = the
// 2-norm of what the two BF16 parts leave out of C_c (exact: the split's differences are exact
// in FP32); one wave per centroid.
__global__ void k_centroid_norms(const float* C, int k, int d, int kp, double* cn) {
  const int c = blockIdx.x;
  double q = 0.0, rq = 0.0;
  if (c < k)
    for (int col = threadIdx.x; col < d; col += 64) {
      const float x = C[static_cast<int64_t>(c) * d + col];
      uint16_t h, m, l;
      split3(x, h, m, l);
      const double v = static_cast<double>(x);
      const double r = (v - static_cast<double>(bf16_to_f32(h))) - static_cast<double>(bf16_to_f32(m));
      q += v * v;
      rq += r * r;
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    q += __shfl_xor(q, off, 64);
    rq += __shfl_xor(rq, off, 64);
  }
  if (threadIdx.x == 0) {
    cn[c] = c < k ? q : INFINITY;
    cn[kp + c] = sqrt(rq);
  }
}

// eight consecutive values of row `row` from column col (zeros past d or n)
template <typename TF>
__device__ inline void load8(const TF* F, int64_t ldf, int64_t n, int d, int64_t row, int col,
                             float* v) {
  if (row < n && col + 8 <= d) {
    const TF* p = F + row * ldf + col;
    if constexpr (sizeof(TF) == 4) {
      const uint4 u0 = reinterpret_cast<const uint4*>(p)[0];
      const uint4 u1 = reinterpret_cast<const uint4*>(p)[1];
      v[0] = __uint_as_float(u0.x); v[1] = __uint_as_float(u0.y);
      v[2] = __uint_as_float(u0.z); v[3] = __uint_as_float(u0.w);
      v[4] = __uint_as_float(u1.x); v[5] = __uint_as_float(u1.y);
      v[6] = __uint_as_float(u1.z); v[7] = __uint_as_float(u1.w);
    } else {
      const uint4 u = reinterpret_cast<const uint4*>(p)[0];
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[2 * i] = __uint_as_float(w[i] << 16);
        v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = (row < n && col + i < d) ? to_f<TF>(F[row * ldf + col + i]) : 0.f;
  }
}

// Raw 16-byte loads of eight consecutive values of row `row` from column col (zeros past d
// or n); RW = 1 (BF16) or 2 (FP32) vectors.  FULL (aligned rows, d a multiple of 8): one
// unmasked load from an in-bounds address, so the loads of a panel stay in flight together;
// rows past n then hold row 0's values (their results are never written) and pieces past d
// are zeroed.
template <typename TF, bool FULL>
__device__ inline void load_raw8(const TF* F, int64_t ldf, int64_t n, int d, int64_t row, int col,
                                 u32x4* raw) {
  constexpr int RW = sizeof(TF) / 2;
  if constexpr (FULL) {
    const u32x4* p = reinterpret_cast<const u32x4*>(F + (row < n ? row : 0) * ldf + (col < d ? col : 0));
    const u32x4 z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const u32x4 v = p[q];
      raw[q] = col < d ? v : z;
    }
    return;
  }
  if (row < n && col + 8 <= d) {
    const u32x4* p = reinterpret_cast<const u32x4*>(F + row * ldf + col);
#pragma unroll
    for (int q = 0; q < RW; ++q) raw[q] = p[q];
  } else {
    TF tmp[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) tmp[i] = (row < n && col + i < d) ? F[row * ldf + col + i] : TF(0);
    __builtin_memcpy(raw, tmp, sizeof(tmp));
  }
}

template <typename TF>
__device__ inline void raw8_to_f(const u32x4* raw, float* v) {
  if constexpr (sizeof(TF) == 4) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[4 * q + i] = __uint_as_float(raw[q][i]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = __uint_as_float(raw[0][i] << 16);
      v[2 * i + 1] = __uint_as_float(raw[0][i] & 0xffff0000u);
    }
  }
}

__device__ inline bf16x8 lds_bf8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

template <typename V>
__device__ inline bool sc_less(V va, int ia, V vb, int ib) {
  return va < vb || (va == vb && ia < ib);
}

// insert (v, i) into the sorted list b[0..2]
template <typename V>
__device__ inline void top3_insert(V* b, int* ix, V v, int i) {
  if (sc_less(v, i, b[2], ix[2])) {
    if (sc_less(v, i, b[1], ix[1])) {
      b[2] = b[1]; ix[2] = ix[1];
      if (sc_less(v, i, b[0], ix[0])) { b[1] = b[0]; ix[1] = ix[0]; b[0] = v; ix[0] = i; }
      else { b[1] = v; ix[1] = i; }
    } else {
      b[2] = v; ix[2] = i;
    }
  }
}

// LDS layout of one staged chunk: kCParts parts x kc_max rows of SB = DP + 8 bf16, then
// kc_max 16-byte records of FP32 norm terms.
template <int DP>
__host__ __device__ constexpr int mf_sb() { return DP + 8; }

inline size_t mf_lds_bytes(int DP, int kc_max) {
  return static_cast<size_t>(kCParts) * kc_max * (DP + 8) * 2 + static_cast<size_t>(kc_max) * 16;
}

// T row tiles per wave and WV waves per block (T > 1 and WV = 8 when the centroids need
// several LDS chunks: each staged chunk then serves 16 WV T rows, dividing the re-staging
// traffic; the registers of T = 2 allow one such block per CU, the same eight waves as two
// blocks of four).
// The one-tile kernels up to 128 columns are held to four waves per SIMD (at most 128
// registers, no spills): the latency of their row loads and LDS reads needs the waves.
template <typename TF, int DP, int T, int WV, bool FULL>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(T == 1 && DP <= 128 ? 4 : 1)))
void k_assign_mf(const TF* F, int64_t ldf, int64_t n, int d,
                                                   const uint16_t* parts, const double* cn_g,
                                                   const float* C, int k, int kp, int kc_max,
                                                   int32_t* labels, float* best_d2,
                                                   double* obj_part) {
  constexpr int SB = mf_sb<DP>();
  constexpr int NS = DP / 32;                      // 32-column MFMA steps
  constexpr int NP = sizeof(TF) == 4 ? 3 : 1;      // BF16 parts of a feature value
  // rounding of one group's FP32 sum of 32 kGroup products, of summing the at most 8 / kGroup
  // groups, and 5 u for the small cross products and the dropped products of the row parts
  // (72 u for pairs); the centroid's dropped part enters through its own norm
  constexpr double E2 = 2.0 * (32.0 * kGroup + (8 / kGroup - 1) + 5) * 0x1p-24 * (1.0 + 0x1p-16);
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint16_t* s_cb = reinterpret_cast<uint16_t*>(s_raw);
  // per staged centroid: FP32 ||c||^2, ||c|| rounded up, and the score's centroid-only
  // half-width term (one 16-byte LDS read per score)
  float4* s_cq = reinterpret_cast<float4*>(s_raw + static_cast<size_t>(kCParts) * kc_max * SB * 2);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int nchunks = (kp + kc_max - 1) / kc_max;
  const int64_t panels = (n + 16 * WV * T - 1) / (16 * WV * T);
  // centroid rows readable as 16-byte pieces
  const bool cvec = d % 4 == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
  const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
  double objsum = 0.0;
  bool staged = false;
  constexpr int RW = sizeof(TF) / 2;
  // BF16 rows, one tile: the next panel's row is prefetched while the current one is scored
  // (FP32 rows already hold three split parts in registers; a prefetch costs occupancy there)
  constexpr bool PF = sizeof(TF) == 2 && T == 1;
  auto row_of = [&](int64_t panel, int t) -> int64_t {
    return ((panel * WV + wave) * T + t) * 16 + li;
  };
  u32x4 raw[T][NS][RW];
  if constexpr (PF) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      load_raw8<TF, FULL>(F, ldf, n, d, row_of(blockIdx.x, 0), s * 32 + lq * 8, raw[0][s]);
  }
  for (int64_t panel = blockIdx.x; panel < panels; panel += gridDim.x) {
    if constexpr (!PF) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s)
          load_raw8<TF, FULL>(F, ldf, n, d, row_of(panel, t), s * 32 + lq * 8, raw[t][s]);
    }
    // three smallest lower ends, smallest upper end, and the row's factors of the half-width
    float bl3[T][3], um[T], gfn[T], rfn[T];
    int bi3[T][3];
    // B operand: row li, eight consecutive columns per step from 8 lq
    bf16x8 a[T][NP][NS];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      um[t] = INFINITY;
#pragma unroll
      for (int q = 0; q < 3; ++q) { bl3[t][q] = INFINITY; bi3[t][q] = 0x7fffffff; }
      float fs = 0.f;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        float v[8];
        raw8_to_f<TF>(raw[t][s], v);
        // BF16 rows are their own operand: the loaded bits, in memory order
        if constexpr (NP == 1) a[t][0][s] = __builtin_bit_cast(bf16x8, raw[t][s][0]);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          fs = fmaf(v[e], v[e], fs);
          if constexpr (NP == 3) {
            uint16_t h, m, l;
            split3(v[e], h, m, l);
            a[t][0][s][e] = __builtin_bit_cast(__bf16, h);
            a[t][1][s][e] = __builtin_bit_cast(__bf16, m);
            a[t][2][s][e] = __builtin_bit_cast(__bf16, l);
          }
        }
      }
      fs += __shfl_xor(fs, 16, 64);
      fs += __shfl_xor(fs, 32, 64);
      // ||f|| bounded above (the FP32 sum of at most 256 squares errs by at most 2^-16)
      const double fnl = sqrt(static_cast<double>(fs)) * (1.0 + 0x1p-16);
      // a score's half-width: (E2 + 16 u) ||f|| ||c|| + 2 ||f|| ||r_c|| + 8 u ||c||^2 + 2^-110
      // (r_c what the centroid's two parts leave out); the u terms cover the FP32 rounding of
      // the score and of its ends, the last any underflow
      gfn[t] = static_cast<float>((E2 + 16.0 * 0x1p-24) * fnl * (1.0 + 0x1p-20));
      rfn[t] = static_cast<float>(fnl * (1.0 + 0x1p-20));
    }
    if (PF && panel + gridDim.x < panels) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        load_raw8<TF, FULL>(F, ldf, n, d, row_of(panel + gridDim.x, 0), s * 32 + lq * 8, raw[0][s]);
    }
    for (int chunk = 0; chunk < nchunks; ++chunk) {
      const int c0 = chunk * kc_max;
      const int kc = min(kc_max, kp - c0);
      if (nchunks > 1 || !staged) {
        __syncthreads();
        // 16-byte copies of the chunk's kCParts parts, SU loads in flight per thread (the last
        // group re-reads the final piece instead of branching), then its norms.  A part's
        // chunk is contiguous in global memory (piece q at 8 q); in LDS its rows are padded
        // to SB, so piece q goes to row q / vpr (a shift: vpr is a power of two).
        constexpr int SU = 4;
        constexpr int vpr = DP / 8;
        const int per = kc * vpr;
#pragma unroll
        for (int pp = 0; pp < kCParts; ++pp) {
          const uint16_t* src = parts + (static_cast<int64_t>(pp) * kp + c0) * DP;
          uint16_t* dst = s_cb + pp * kc_max * SB;
          for (int q0 = threadIdx.x; q0 < per; q0 += SU * blockDim.x) {
            u32x4 val[SU];
#pragma unroll
            for (int j = 0; j < SU; ++j) {
              const int q = min(q0 + j * static_cast<int>(blockDim.x), per - 1);
              val[j] = *reinterpret_cast<const u32x4*>(src + 8 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < SU; ++j) {
              const int q = q0 + j * static_cast<int>(blockDim.x);
              if (q < per)
                *reinterpret_cast<u32x4*>(dst + (q / vpr) * SB + 8 * (q % vpr)) = val[j];
            }
          }
        }
        for (int c = threadIdx.x; c < kc; c += blockDim.x) {
          const double q = cn_g[c0 + c];
          s_cq[c] = make_float4(static_cast<float>(q), static_cast<float>(sqrt(q) * (1.0 + 0x1p-20)),
                                static_cast<float>(8.0 * 0x1p-24 * q * (1.0 + 0x1p-20) + 0x1p-110),
                                static_cast<float>(2.0 * cn_g[kp + c0 + c] * (1.0 + 0x1p-20)));
        }
        __syncthreads();
        staged = true;
      }
      for (int ct = 0; ct < kc / 16; ++ct) {
        // A operand: centroid ct*16 + li; output register r of lane (li, lq) is centroid
        // ct*16 + 4 lq + r against row li of the tile
        const uint16_t* cb = s_cb + (ct * 16 + li) * SB + lq * 8;
        // every pair of steps starts its own accumulators, so the matrix-core chains are at
        // most four long and the pairs overlap in the pipeline (one chain across all steps
        // runs slower: each product then waits for the previous one); a pair's leading and
        // small products are then added to two running FP32 sums.  A step's three centroid
        // fragments are read from LDS once for all T row tiles, and the next step's are
        // requested before this step's products, so the reads' latency hides behind them.
        f32x4 dot[T], small[T], pm[T], ps[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          small[t] = zero4;
          dot[t] = zero4;
          pm[t] = zero4;
          ps[t] = zero4;
        }
        bf16x8 ch = lds_bf8(cb), cm = lds_bf8(cb + kc_max * SB);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          bf16x8 nh = ch, nm = cm;
          if (s + 1 < NS) {
            nh = lds_bf8(cb + (s + 1) * 32);
            nm = lds_bf8(cb + kc_max * SB + (s + 1) * 32);
          }
#pragma unroll
          for (int t = 0; t < T; ++t) {
            // steps after a group's first continue its accumulators; the group is then summed
            const bool cont = (s % kGroup) != 0;
            pm[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, a[t][0][s], cont ? pm[t] : zero4, 0, 0, 0);
            ps[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cm, a[t][0][s], cont ? ps[t] : zero4, 0, 0, 0);
            if constexpr (NP == 3) {
              ps[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, a[t][1][s], ps[t], 0, 0, 0);
              ps[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cm, a[t][1][s], ps[t], 0, 0, 0);
              ps[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, a[t][2][s], ps[t], 0, 0, 0);
            }
            if (s % kGroup == kGroup - 1 || s + 1 == NS) {
              small[t] += ps[t];
              dot[t] += pm[t];
            }
          }
          ch = nh;
          cm = nm;
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int lc = ct * 16 + mf_drow(r, lq);
            const int cent = c0 + lc;
            float* b = bl3[t];
            int* ix = bi3[t];
            if constexpr (T == 1 && NP == 1) {
              // sorted insertion of (lo, cent) into the three smallest lower ends, as selects
              // (no branches, so no register shuffling at joins); centroids arrive in
              // increasing index order within a lane, and strict < keeps ties on the lower
              // index
              const float4 cq = s_cq[lc];
              const float sc = fmaf(-2.f, dot[t][r] + small[t][r], cq.x);
              const float e = fmaf(rfn[t], cq.w, fmaf(gfn[t], cq.y, cq.z));
              const bool real = cent < k;
              um[t] = real ? fminf(um[t], sc + e) : um[t];
              const float lo = real ? sc - e : INFINITY;
              const bool l0 = lo < b[0], l1 = lo < b[1], l2 = lo < b[2];
              b[2] = l1 ? b[1] : (l2 ? lo : b[2]);
              ix[2] = l1 ? ix[1] : (l2 ? cent : ix[2]);
              b[1] = l0 ? b[0] : (l1 ? lo : b[1]);
              ix[1] = l0 ? ix[0] : (l1 ? cent : ix[1]);
              b[0] = l0 ? lo : b[0];
              ix[0] = l0 ? cent : ix[0];
            } else if (cent < k) {
              // the same insertion with branches (two row tiles or FP32 rows: the selects'
              // extra live registers would cost occupancy or spill)
              const float4 cq = s_cq[lc];
              const float sc = fmaf(-2.f, dot[t][r] + small[t][r], cq.x);
              const float e = fmaf(rfn[t], cq.w, fmaf(gfn[t], cq.y, cq.z));
              um[t] = fminf(um[t], sc + e);
              const float lo = sc - e;
              if (lo < b[2]) {
                if (lo < b[1]) {
                  b[2] = b[1]; ix[2] = ix[1];
                  if (lo < b[0]) { b[1] = b[0]; ix[1] = ix[0]; b[0] = lo; ix[0] = cent; }
                  else { b[1] = lo; ix[1] = cent; }
                } else {
                  b[2] = lo; ix[2] = cent;
                }
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t row = row_of(panel, t);
      const bool valid = row < n;
      float* b = bl3[t];
      int* ix = bi3[t];
      // merge over the four lanes of the row (lq), in (value, index) order
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        float ob[3];
        int oi[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) { ob[q] = __shfl_xor(b[q], off, 64); oi[q] = __shfl_xor(ix[q], off, 64); }
#pragma unroll
        for (int q = 0; q < 3; ++q) top3_insert(b, ix, ob[q], oi[q]);
        um[t] = fminf(um[t], __shfl_xor(um[t], off, 64));
      }
      // candidates: lower end not above the smallest upper end (the first always is)
      const bool certain = !valid || ix[1] >= k || b[1] > um[t];
      const bool pair = !certain && (ix[2] >= k || b[2] > um[t]);
      int lab = ix[0] < k ? ix[0] : 0;  // (no candidate only with NaN features)
      double best = 0.0;
      // FP64 squared distance from the row to centroid c (the direct form): each lane covers
      // the columns s * 32 + 8 lq + i of the row (just read, so cached) and of the centroid,
      // SG 32-column steps per round with their loads in flight together (two in the one-tile
      // kernels, whose registers are kept for occupancy); the four lanes of the row then add
      // their sums.
      auto dist_to = [&](int c) -> double {
        const float* crow = C + static_cast<int64_t>(c) * d;
        constexpr int SG0 = T == 1 ? 2 : 4;
        constexpr int SG = NS < SG0 ? NS : SG0;
        double e = 0.0;
#pragma unroll 1
        for (int s0 = 0; s0 < NS; s0 += SG) {
          u32x4 fr[SG][RW];
          float cv[SG][8];
#pragma unroll
          for (int g = 0; g < SG; ++g) {
            const int col0 = (s0 + g) * 32 + lq * 8;
            load_raw8<TF, FULL>(F, ldf, n, d, row, col0, fr[g]);
            if (cvec && col0 + 8 <= d) {
              const float4 u0 = reinterpret_cast<const float4*>(crow + col0)[0];
              const float4 u1 = reinterpret_cast<const float4*>(crow + col0)[1];
              cv[g][0] = u0.x; cv[g][1] = u0.y; cv[g][2] = u0.z; cv[g][3] = u0.w;
              cv[g][4] = u1.x; cv[g][5] = u1.y; cv[g][6] = u1.z; cv[g][7] = u1.w;
            } else {
#pragma unroll
              for (int q = 0; q < 8; ++q) cv[g][q] = col0 + q < d ? crow[col0 + q] : 0.f;
            }
          }
#pragma unroll
          for (int g = 0; g < SG; ++g) {
            float fv[8];
            raw8_to_f<TF>(fr[g], fv);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const double tv = static_cast<double>(fv[q]) - static_cast<double>(cv[g][q]);
              e += tv * tv;
            }
          }
        }
        e += __shfl_xor(e, 16, 64);
        e += __shfl_xor(e, 32, 64);
        return e;
      };
      if (!certain) {
        // the direct form against the candidates: the two best, else every centroid
        double be = INFINITY;
        int bl = 0x7fffffff;
        if (pair) {
          const double e0 = dist_to(ix[0]), e1 = dist_to(ix[1]);
          if (sc_less(e0, ix[0], be, bl)) { be = e0; bl = ix[0]; }
          if (sc_less(e1, ix[1], be, bl)) { be = e1; bl = ix[1]; }
        } else {
          for (int c = 0; c < k; ++c) {
            const double e = dist_to(c);
            if (sc_less(e, c, be, bl)) { be = e; bl = c; }
          }
        }
        lab = bl;
        best = be;
      } else if (valid && (best_d2 || obj_part)) {
        best = dist_to(lab);
      }
      if (valid && lq == 0) {
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

__global__ void k_upd_clear(int32_t* cnt, int k, uint32_t* maxabs) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < k) cnt[t] = 0;
  if (t == 0 && maxabs) maxabs[0] = 0u;
}

// max |F| as float bits (the fixed-point scale of the update).  A contiguous, 16-byte aligned
// block is read as one flat array of 16-byte pieces; otherwise row by row.
template <typename TF>
__global__ void k_maxabs(const TF* F, int64_t ldf, int64_t n, int d, int flat, uint32_t* out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  float m = 0.f;
  if (flat) {
    constexpr int V = 16 / sizeof(TF);
    const int64_t total = n * d, nv = total / V;
    const uint4* P = reinterpret_cast<const uint4*>(F);
    for (int64_t i = gid; i < nv; i += stride) {
      const uint4 u = P[i];
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (sizeof(TF) == 4) {
          m = fmaxf(m, fabsf(__uint_as_float(w[q])));
        } else {
          m = fmaxf(m, fabsf(__uint_as_float(w[q] << 16)));
          m = fmaxf(m, fabsf(__uint_as_float(w[q] & 0xffff0000u)));
        }
      }
    }
    for (int64_t i = nv * V + gid; i < total; i += stride) m = fmaxf(m, fabsf(to_f<TF>(F[i])));
  } else {
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x)
      for (int c = threadIdx.x; c < d; c += blockDim.x) m = fmaxf(m, fabsf(to_f<TF>(F[r * ldf + c])));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// The update orders the rows by label with a counting sort (label counts, their prefix sums,
// a scatter of row indices), then sums each label's rows in chunks of kUpdChunk: one block
// per chunk, whose rows all carry the chunk's label, so a block keeps one running sum per
// column in registers and writes one 64-bit partial sum per column.  A last pass adds each
// label's chunk partials in chunk order.  All sums are 64-bit fixed point, so neither the
// order of the rows within a label nor the grouping changes them.
constexpr int kUpdChunk = 512;       // rows per chunk (the last chunk of a label may be short)
constexpr int kUpdScatterRows = 8192;  // rows per scatter block (one global atomic per label each)

// Label counts (out-of-range labels are ignored): an LDS histogram per block, then one global
// atomic per label.
__global__ __launch_bounds__(kThreads) void k_lab_hist(const int32_t* labels, int64_t n, int k,
                                                       int32_t* cnt) {
  __shared__ int32_t h[256];
  for (int t = threadIdx.x; t < k; t += kThreads) h[t] = 0;
  __syncthreads();
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const int32_t lb = labels[i];
    if (lb >= 0 && lb < k) atomicAdd(&h[lb], 1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += kThreads)
    if (h[t]) atomicAdd(&cnt[t], h[t]);
}

// One block: off[c] = rows with a smaller label, cur[c] = off[c] (the scatter's cursor), and
// first[c] = chunks of the smaller labels; first[k] = all chunks, off[k] = all valid rows.
__global__ __launch_bounds__(kThreads) void k_lab_scan(const int32_t* cnt, int k, int32_t* off,
                                                       int32_t* cur, int32_t* first) {
  __shared__ int32_t s_w[2][kThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int c = t < k ? cnt[t] : 0;
  const int ch = (c + kUpdChunk - 1) / kUpdChunk;
  int x = c, y = ch;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xa = __shfl_up(x, o, 64), ya = __shfl_up(y, o, 64);
    if (lane >= o) { x += xa; y += ya; }
  }
  if (lane == 63) { s_w[0][wave] = x; s_w[1][wave] = y; }
  __syncthreads();
  int ax = 0, ay = 0;
  for (int w = 0; w < wave; ++w) { ax += s_w[0][w]; ay += s_w[1][w]; }
  if (t < k) {
    off[t] = ax + x - c;
    cur[t] = ax + x - c;
    first[t] = ay + y - ch;
  }
  if (t == k - 1) {
    off[k] = ax + x;
    first[k] = ay + y;
  }
}

// Scatter: block b takes rows [b * kUpdScatterRows, ...), reserves a range of each label's
// slots with one global atomic per label, and writes each row's index into it.
__global__ __launch_bounds__(kThreads) void k_lab_scatter(const int32_t* labels, int64_t n, int k,
                                                          int32_t* cur, int32_t* perm) {
  constexpr int PER = kUpdScatterRows / kThreads;
  __shared__ int32_t h[256];
  __shared__ int32_t base[256];
  for (int t = threadIdx.x; t < k; t += kThreads) h[t] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kUpdScatterRows;
  int32_t lb[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int64_t r = r0 + i * kThreads + threadIdx.x;
    lb[i] = r < n ? labels[r] : -1;
    if (lb[i] < 0 || lb[i] >= k) lb[i] = -1;
    if (lb[i] >= 0) atomicAdd(&h[lb[i]], 1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += kThreads) {
    base[t] = h[t] ? atomicAdd(&cur[t], h[t]) : 0;
    h[t] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (lb[i] >= 0)
      perm[base[lb[i]] + atomicAdd(&h[lb[i]], 1)] = static_cast<int32_t>(r0 + i * kThreads + threadIdx.x);
}

// Chunk sums: block b (< first[k]) takes chunk b, whose rows all have the label c with
// first[c] <= b < first[c + 1].  A row is covered by LR lanes of 8 columns each (LR a power
// of two, 8 LR >= d); the kThreads / LR row groups of the block take the chunk's rows in turn
// and their sums meet in LDS in group order.  Writes part[b * d + col] for col < d.
template <typename TF, bool VEC, int LR>
__global__ __launch_bounds__(kThreads) void k_lab_sum(const TF* F, int64_t ldf, int64_t n, int d,
                                                      int k, const int32_t* off,
                                                      const int32_t* first, const int32_t* perm,
                                                      const uint32_t* maxabs,
                                                      unsigned long long* part) {
  constexpr int G = kThreads / LR;  // row groups
  __shared__ int32_t s_rows[kUpdChunk];
  __shared__ long long s_red[kThreads * 8];
  const int32_t b = static_cast<int32_t>(blockIdx.x);
  if (b >= first[k]) return;  // (uniform across the block)
  int lo = 0, hi = k - 1;     // the label whose chunks include b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int32_t p0 = off[lo] + (b - first[lo]) * kUpdChunk;
  const int nr = min(kUpdChunk, off[lo + 1] - p0);
  for (int i = threadIdx.x; i < nr; i += kThreads) s_rows[i] = perm[p0 + i];
  __syncthreads();

  const float mxf = __uint_as_float(maxabs[0]);
  const int S = fixed_scale(mxf, n);
  int em = 0;
  frexpf(mxf, &em);
  const int hb = em + S;  // every converted value is an integer of magnitude <= 2^hb
  const int g = threadIdx.x / LR;
  const int c8 = (threadIdx.x % LR) * 8;
  // VEC (aligned rows, d a multiple of 8): unmasked 16-byte loads; a lane past d reads
  // column 0 and its sums are never written
  const int lcol = VEC && c8 >= d ? 0 : c8;
  constexpr int RW = sizeof(TF) / 2;  // 16-byte pieces per eight values
  auto load_raw = [&](int32_t row, uint4* raw) {
    const TF* rp = F + static_cast<int64_t>(row) * ldf + lcol;
    if constexpr (VEC) {
#pragma unroll
      for (int w = 0; w < RW; ++w) raw[w] = reinterpret_cast<const uint4*>(rp)[w];
    } else {
      TF tmp[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) tmp[i] = c8 + i < d ? rp[i] : TF(0);
      __builtin_memcpy(raw, tmp, sizeof(tmp));
    }
  };
  auto unpack = [&](const uint4* raw, float* v) {
    if constexpr (sizeof(TF) == 4) {
      v[0] = __uint_as_float(raw[0].x); v[1] = __uint_as_float(raw[0].y);
      v[2] = __uint_as_float(raw[0].z); v[3] = __uint_as_float(raw[0].w);
      v[4] = __uint_as_float(raw[1].x); v[5] = __uint_as_float(raw[1].y);
      v[6] = __uint_as_float(raw[1].z); v[7] = __uint_as_float(raw[1].w);
    } else {
      const uint32_t w[4] = {raw[0].x, raw[0].y, raw[0].z, raw[0].w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[2 * i] = __uint_as_float(w[i] << 16);
        v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
      }
    }
  };
  long long sum[8];
  // A group sums at most ceil(nr / G) values per column.  When that many values of
  // magnitude <= 2^hb stay within 2^53, every partial sum is an integer that FP64 holds
  // exactly: each value is then rounded to an integer in FP32 (v * 2^S is exact there, and
  // rintf rounds half to even like llrint) and summed in FP64, converted to 64 bits once at
  // the end.  Otherwise each value is converted to 64 bits on its own.  Both give the same
  // integers.
  auto walk = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    using Acc = std::conditional_t<FAST, double, long long>;
    Acc acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0;
    auto add = [&](const float* v) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (FAST) acc[i] += static_cast<double>(rintf(ldexpf(v[i], S)));
        else acc[i] += llrint(ldexp(static_cast<double>(v[i]), S));
      }
    };
    // UR rows in flight per lane (eight 16-byte loads)
    constexpr int UR = 8 / RW;
    int q = g;
    for (; q + (UR - 1) * G < nr; q += UR * G) {
      uint4 raw[UR][RW];
#pragma unroll
      for (int u = 0; u < UR; ++u) load_raw(s_rows[q + u * G], raw[u]);
      // all the rows' loads ahead of the first use
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        float v[8];
        unpack(raw[u], v);
        add(v);
      }
    }
    for (; q < nr; q += G) {
      uint4 raw[RW];
      load_raw(s_rows[q], raw);
      float v[8];
      unpack(raw, v);
      add(v);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) sum[i] = static_cast<long long>(acc[i]);
  };
  const int per = (nr + G - 1) / G;
  if (hb <= 53 && (53 - hb >= 30 || per <= (1 << (53 - hb)))) walk(std::true_type{});
  else walk(std::false_type{});
#pragma unroll
  for (int i = 0; i < 8; ++i) s_red[(g * LR + threadIdx.x % LR) * 8 + i] = sum[i];
  __syncthreads();
  // thread t < 8 LR adds column t over the groups, in group order
  if (threadIdx.x < LR * 8 && static_cast<int>(threadIdx.x) < d) {
    const int lane = threadIdx.x / 8, i = threadIdx.x % 8;
    long long t = 0;
    for (int gg = 0; gg < G; ++gg) t += s_red[(gg * LR + lane) * 8 + i];
    part[static_cast<int64_t>(b) * d + threadIdx.x] = static_cast<unsigned long long>(t);
  }
}

// Per (c, col): the sum of label c's chunk partials (integers: any order gives the same
// value), then C[c] = sum / count (C may be null), sums_out = the sum rounded once to FP32
// (or null), counts = the cluster sizes (or null).
__global__ void k_upd_final(const unsigned long long* part, const int32_t* first,
                            const int32_t* gcnt, const uint32_t* maxabs, int64_t n, int k, int d,
                            float* C, int32_t* counts, float* sums_out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(k) * d) return;
  const int c = static_cast<int>(t / d), col = static_cast<int>(t % d);
  const int32_t j0 = first[c], j1 = first[c + 1];
  unsigned long long a[4] = {0ull, 0ull, 0ull, 0ull};
  int32_t j = j0;
  for (; j + 4 <= j1; j += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] += part[static_cast<int64_t>(j + q) * d + col];
  }
  for (; j < j1; ++j) a[0] += part[static_cast<int64_t>(j) * d + col];
  const unsigned long long tot = a[0] + a[1] + a[2] + a[3];
  const int S = fixed_scale(__uint_as_float(maxabs[0]), n);
  const int32_t cnt = gcnt[c];
  const double sum = ldexp(static_cast<double>(static_cast<long long>(tot)), -S);
  if (C && cnt > 0) C[t] = static_cast<float>(sum / static_cast<double>(cnt));
  if (sums_out) sums_out[t] = static_cast<float>(sum);
  if (counts && col == 0) counts[c] = cnt;
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

// cd[a] = ||C_cj - C_a||^2 (FP64) for the earlier centres a < cj; one wave per centre,
// lanes over the columns, fixed shuffle tree.
__global__ void k_pp_cdist(const float* C, int d, int cj, double* cd) {
  const int a = blockIdx.x;
  double q = 0.0;
  for (int t = threadIdx.x; t < d; t += 64) {
    const double v = static_cast<double>(C[static_cast<int64_t>(cj) * d + t]) -
                     static_cast<double>(C[static_cast<int64_t>(a) * d + t]);
    q += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
  if (threadIdx.x == 0) cd[a] = q;
}

// d2[i] = min(d2[i], ||f_i - C_cj||^2) in FP64 (first round: the distance itself), owner[i]
// = the centre that attains it.  Block b covers the contiguous rows [b * kThreads * kRIT, ...)
// and writes their sum to bsum[b].  A row is skipped without reading it when
// ||C_cj - C_owner||^2 >= 4 d2 (1 + 1e-9): by the triangle inequality the new centre is then
// no closer, so the result equals the unpruned pass (the margin covers the FP64 rounding of
// both sides).  The block first reads the current distances and owners of all its rows
// (coalesced), decides which rows to read and lists them in row order, so the feature loads
// that follow wait on no other global load and a pruned row costs no instruction beyond its
// test.  Sixteen lanes share a listed row so that each load instruction reads whole rows; the
// lanes' partial sums meet in a fixed shuffle tree.  The block's sum of the new distances is
// taken over all its rows in a fixed order.
template <typename TF, bool VEC, int NPC>
__global__ __launch_bounds__(kThreads) void k_pp_dist(const TF* F, int64_t ldf, int64_t n, int d,
                                                      int dp, const float* C, int cj, int first,
                                                      const double* cd, int32_t* owner,
                                                      double* d2, double* bsum) {
  constexpr int V = 16 / sizeof(TF);  // values per 16-byte piece; a lane reads NPC pieces
  constexpr int U = VEC ? 8 / NPC : 2;  // rows per group in flight
  constexpr int RB = kThreads * kRIT;  // rows per block
  __shared__ float s_cj[256];
  __shared__ double s_cd[256];
  __shared__ double s_old[RB];
  __shared__ unsigned char s_need[RB];
  const float* Cj = C + static_cast<int64_t>(cj) * d;
  for (int t = threadIdx.x; t < dp; t += kThreads) s_cj[t] = t < d ? Cj[t] : 0.f;
  if (!first)
    for (int t = threadIdx.x; t < cj; t += kThreads) s_cd[t] = cd[t];
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RB;
  if (first) {
#pragma unroll
    for (int i = 0; i < kRIT; ++i) {
      const int r = threadIdx.x + i * kThreads;
      s_old[r] = 0.0;
      s_need[r] = base + r < n ? 1 : 0;
    }
  } else {
    double dv[kRIT];
    int32_t ow[kRIT];
#pragma unroll
    for (int i = 0; i < kRIT; ++i) {
      const int64_t row = base + threadIdx.x + i * kThreads;
      const int64_t rr = row < n ? row : n - 1;  // rows past n read the last row, unused
      dv[i] = d2[rr];
      ow[i] = owner[rr];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < kRIT; ++i) {
      const int r = threadIdx.x + i * kThreads;
      const bool in = base + r < n;
      s_old[r] = in ? dv[i] : 0.0;
      s_need[r] = (in && !(s_cd[ow[i]] >= 4.0 * dv[i] * (1.0 + 1e-9))) ? 1 : 0;
    }
  }
  __syncthreads();
  const int l16 = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;  // 16 row groups per block
  double cjd[NPC][V];  // the lane's columns of the new centre
#pragma unroll
  for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int c = (pc * 16 + l16) * V + i;
      cjd[pc][i] = c < d ? static_cast<double>(s_cj[c]) : 0.0;
    }
  // the rows to read, in row order: a wave ballot per stretch of kThreads rows
  __shared__ int16_t s_list[RB];
  __shared__ int s_wcnt[kThreads / 64];
  __shared__ int s_total;
  if (threadIdx.x == 0) s_total = 0;
  __syncthreads();
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kRIT; ++i) {
      const int r = threadIdx.x + i * kThreads;
      const bool nd = s_need[r] != 0;
      const uint64_t bal = __ballot(nd);
      const int before = __popcll(bal & ((uint64_t(1) << lane) - 1));
      if (lane == 0) s_wcnt[wave] = __popcll(bal);
      __syncthreads();
      int off = s_total;
      for (int w = 0; w < wave; ++w) off += s_wcnt[w];
      if (nd) s_list[off + before] = static_cast<int16_t>(r);
      __syncthreads();
      if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) s_total += s_wcnt[w];
      __syncthreads();
    }
  }
  const int cnt = s_total;
  for (int q0 = 0; q0 < cnt; q0 += 16 * U) {
    uint4 raw[U][NPC];
    bool need[U];
    int rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int li = q0 + u * 16 + grp;
      need[u] = li < cnt;
      rr[u] = need[u] ? s_list[li] : 0;
      const int64_t row = base + rr[u];
      if constexpr (VEC) {
        // branch-free, so that all U x NPC loads are in flight together: list slots past the
        // end read row 0 and pieces past d read column 0 (in bounds, cached, and never used)
        const TF* rowp = F + (need[u] ? row : 0) * ldf;
#pragma unroll
        for (int pc = 0; pc < NPC; ++pc) {
          const int c0 = (pc * 16 + l16) * V;
          raw[u][pc] = *reinterpret_cast<const uint4*>(rowp + (c0 < d ? c0 : 0));
        }
      } else {
        const TF* rowp = F + (need[u] ? row : 0) * ldf;
#pragma unroll
        for (int pc = 0; pc < NPC; ++pc) {
          const int c0 = (pc * 16 + l16) * V;
          TF tmp[V];
#pragma unroll
          for (int i = 0; i < V; ++i) tmp[i] = (need[u] && c0 + i < d) ? rowp[c0 + i] : TF(0);
          __builtin_memcpy(&raw[u][pc], tmp, 16);
        }
      }
    }
    // keep the loads of all U rows ahead of the first use
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = base + rr[u];
      double s = 0.0;
#pragma unroll
      for (int pc = 0; pc < NPC; ++pc) {
        const int c0 = (pc * 16 + l16) * V;
        const uint32_t w[4] = {raw[u][pc].x, raw[u][pc].y, raw[u][pc].z, raw[u][pc].w};
        float f[V];
        if constexpr (sizeof(TF) == 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i) f[i] = __uint_as_float(w[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
          }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
          // columns past d add an exact zero
          const double t = c0 + i < d ? static_cast<double>(f[i]) - cjd[pc][i] : 0.0;
          s += t * t;
        }
      }
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 16);
      if (need[u] && l16 == 0) {
        if (first) {
          s_old[rr[u]] = s;
          d2[row] = s;
          owner[row] = 0;
        } else if (s < s_old[rr[u]]) {
          s_old[rr[u]] = s;
          d2[row] = s;
          owner[row] = cj;
        }
      }
    }
  }
  __syncthreads();
  // the block's sum of the (new) distances, each thread's rows in order, then a fixed tree
  double local = 0.0;
#pragma unroll
  for (int i = 0; i < kRIT; ++i) local += s_old[threadIdx.x + i * kThreads];
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

csc_status launch_maxabs(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                         uint32_t* mx, hipStream_t s) {
  const int flat = (ldf == d && reinterpret_cast<uintptr_t>(F) % 16 == 0) ? 1 : 0;
  const unsigned mblocks = static_cast<unsigned>(
      std::max<int64_t>(1, std::min<int64_t>(2048, flat ? (n * d / 8 + 255) / 256 : n)));
  if (f_dt == CSC_F32)
    hipLaunchKernelGGL(k_maxabs<float>, dim3(mblocks), dim3(256), 0, s, static_cast<const float*>(F),
                       ldf, n, d, flat, mx);
  else
    hipLaunchKernelGGL(k_maxabs<uint16_t>, dim3(mblocks), dim3(256), 0, s,
                       static_cast<const uint16_t*>(F), ldf, n, d, flat, mx);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

int64_t assign_blocks(int64_t n) {
  const int64_t per = static_cast<int64_t>(kThreads) * kRIT;
  return std::max<int64_t>(1, (n + per - 1) / per);
}

struct KmLayout {
  size_t off_u, off_d2, off_bsum, off_cnt, off_max, off_obj, off_objv, off_sel, off_cp,
      off_own, off_cd, off_perm, off_part, off_tab, total;
};

// chunks of the update's label-ordered rows: at most one short chunk per label
int64_t upd_chunks(int64_t n, int k) { return (n + kUpdChunk - 1) / kUpdChunk + k; }

int padded_k(int k) { return (k + kKG - 1) / kKG * kKG; }

KmLayout km_layout(int64_t n, int d, int k) {
  KmLayout L{};
  const int64_t blocks = assign_blocks(n);
  size_t off = 0;
  L.off_u = off; off += align_up(static_cast<size_t>(k) * 8);
  L.off_d2 = off; off += align_up(static_cast<size_t>(n) * 8);
  L.off_bsum = off; off += align_up(static_cast<size_t>(blocks) * 8);
  L.off_cnt = off; off += align_up(static_cast<size_t>(k) * 4);
  L.off_max = off; off += 256;
  L.off_obj = off; off += align_up(static_cast<size_t>(std::max<int64_t>(blocks, 2048)) * 8);
  L.off_objv = off; off += align_up(static_cast<size_t>(1024 + 1) * 8);
  L.off_sel = off; off += 256;
  L.off_cp = off; off += align_up(assign_scratch_bytes(k, d));
  L.off_own = off; off += align_up(static_cast<size_t>(n) * 4);
  L.off_cd = off; off += align_up(static_cast<size_t>(k) * 8);
  L.off_perm = off; off += align_up(static_cast<size_t>(n) * 4);
  L.off_part = off; off += align_up(static_cast<size_t>(upd_chunks(n, k)) * d * 8);
  L.off_tab = off; off += align_up(static_cast<size_t>(k + 1) * 12);
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
  // (the update's label scan takes one thread per label, and its label histograms and the
  // allocation-free assignment's static centroid array are sized for 240 labels)
  if (k > 240) return fail(CSC_E_ARG, "k must be <= 240");
  static_assert(240 <= kThreads, "one scan thread per label");
  return CSC_OK;
}

csc_status update_impl(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                       const int32_t* labels, int k, float* C, int32_t* counts, void* work,
                       bool max_ready, hipStream_t s, float* sums_out = nullptr) {
  if (n > INT32_MAX) return fail(CSC_E_ARG, "the update takes fewer than 2^31 rows");
  const KmLayout L = km_layout(n, d, k);
  char* base = static_cast<char*>(work);
  auto* cnt = reinterpret_cast<int32_t*>(base + L.off_cnt);
  auto* mx = reinterpret_cast<uint32_t*>(base + L.off_max);
  auto* perm = reinterpret_cast<int32_t*>(base + L.off_perm);
  auto* part = reinterpret_cast<unsigned long long*>(base + L.off_part);
  auto* off = reinterpret_cast<int32_t*>(base + L.off_tab);
  int32_t* cur = off + (k + 1);
  int32_t* first = cur + (k + 1);
  const int64_t kd = static_cast<int64_t>(k) * d;
  // the counts start at zero
  hipLaunchKernelGGL(k_upd_clear, dim3(static_cast<unsigned>((k + 255) / 256)), dim3(256), 0, s,
                     cnt, k, max_ready ? nullptr : mx);
  if (!max_ready) CSC_TRY(launch_maxabs(F, f_dt, ldf, n, d, mx, s));
  // few blocks: each adds its k counts with global atomics, which serialise per label
  hipLaunchKernelGGL(k_lab_hist, dim3(static_cast<unsigned>(std::min<int64_t>(256, (n + kThreads - 1) / kThreads))),
                     dim3(kThreads), 0, s, labels, n, k, cnt);
  hipLaunchKernelGGL(k_lab_scan, dim3(1), dim3(kThreads), 0, s, cnt, k, off, cur, first);
  hipLaunchKernelGGL(k_lab_scatter, dim3(static_cast<unsigned>((n + kUpdScatterRows - 1) / kUpdScatterRows)),
                     dim3(kThreads), 0, s, labels, n, k, cur, perm);
  const unsigned chunks = static_cast<unsigned>(upd_chunks(n, k));
  const bool vec = rows_aligned(F, f_dt, ldf) && d % 8 == 0;
  const int lr = d <= 32 ? 4 : d <= 64 ? 8 : d <= 128 ? 16 : 32;
#define CSC_SUM(TF, V, LR)                                                                      \
  hipLaunchKernelGGL((k_lab_sum<TF, V, LR>), dim3(chunks), dim3(kThreads), 0, s,                 \
                     static_cast<const TF*>(F), ldf, n, d, k, off, first, perm, mx, part)
#define CSC_SUM_LR(TF, V)                                                                       \
  switch (lr) {                                                                                 \
    case 4: CSC_SUM(TF, V, 4); break;                                                           \
    case 8: CSC_SUM(TF, V, 8); break;                                                           \
    case 16: CSC_SUM(TF, V, 16); break;                                                         \
    default: CSC_SUM(TF, V, 32); break;                                                         \
  }
  if (f_dt == CSC_F32) {
    if (vec) { CSC_SUM_LR(float, true) } else { CSC_SUM_LR(float, false) }
  } else {
    if (vec) { CSC_SUM_LR(uint16_t, true) } else { CSC_SUM_LR(uint16_t, false) }
  }
#undef CSC_SUM_LR
#undef CSC_SUM
  hipLaunchKernelGGL(k_upd_final, dim3(static_cast<unsigned>((kd + 255) / 256)), dim3(256), 0, s,
                     part, first, cnt, mx, n, k, d, C, counts, sums_out);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace

size_t kmeans_workspace(int64_t n, int d, int k) { return km_layout(n, d, k).total; }

// Launch plan of the MFMA assignment for (n, d, k); DP == 0 when it does not apply (d > 256).
// Chunks of kc centroids fill at most 64 KiB of LDS.  One 16-row tile per wave when all
// centroids fit one chunk (staged once per block); two when they do not (BF16 rows), so that
// each re-staged chunk serves 128 rows.
struct MfPlan {
  int DP = 0, kp = 0, kc = 0, T = 1, wv = 4;
  size_t lds = 0;
  int64_t blocks = 1;
};

MfPlan mf_plan(int64_t n, int d, int k, bool bf16_rows = false) {
  MfPlan P;
  if (d > 256) return P;
  int DP = 32;
  while (DP < d) DP <<= 1;
  const int kp = (k + 15) / 16 * 16;
  int kc = 16;
  while (kc + 16 <= kp && mf_lds_bytes(DP, kc + 16) <= 64 * 1024) kc += 16;
  P.DP = DP;
  P.kp = kp;
  P.kc = kc;
  P.T = (bf16_rows && kc < kp) ? 2 : 1;
  // the two-tile kernel runs one 8-wave block per CU, so its chunks may fill the CU's whole
  // LDS (160 KiB on gfx950): fewer chunks, fewer restaging rounds per panel
  if (P.T == 2)
    while (kc + 16 <= kp && mf_lds_bytes(DP, kc + 16) <= 160 * 1024) kc += 16;
  P.kc = kc;
  P.wv = P.T == 2 ? 8 : 4;
  P.lds = mf_lds_bytes(DP, kc);
  const int64_t panels = (n + 16 * P.wv * P.T - 1) / (16 * P.wv * P.T);
  const int64_t per_cu = P.wv == 8 ? 1 :
      std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / static_cast<int64_t>(P.lds)));
  P.blocks = std::max<int64_t>(1, std::min<int64_t>(panels, 256 * per_cu));
  return P;
}

// centroid scratch of the MFMA assignment: two BF16 parts (kp x DP each), then kp squared
// norms and kp norms of what the parts leave out
size_t mf_scratch_bytes(int k, int d) {
  const MfPlan P = mf_plan(1, d, k);
  if (!P.DP) return 0;
  return align_up(static_cast<size_t>(kCParts) * P.kp * P.DP * 2) + static_cast<size_t>(P.kp) * 16;
}

size_t assign_scratch_bytes(int k, int d) {
  return std::max(static_cast<size_t>(padded_k(k)) * padded_d(d) * 4, mf_scratch_bytes(k, d));
}

int64_t assign_parts(int64_t n, int d, int k, const void* F, csc_dtype f_dt, int64_t ldf) {
  const MfPlan P = mf_plan(n, d, k, f_dt == CSC_BF16);
  return (P.DP && rows_aligned(F, f_dt, ldf)) ? P.blocks : assign_blocks(n);
}

static csc_status assign_impl(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                              const float* C, int k, int32_t* labels, float* best_d2,
                              double* obj_part, float* Cp, hipStream_t s) {
  const MfPlan P = mf_plan(n, d, k, f_dt == CSC_BF16);
  if (P.DP && rows_aligned(F, f_dt, ldf)) {
    auto* parts = reinterpret_cast<uint16_t*>(Cp);
    auto* cn = reinterpret_cast<double*>(reinterpret_cast<char*>(Cp) +
                                         align_up(static_cast<size_t>(kCParts) * P.kp * P.DP * 2));
    hipLaunchKernelGGL(k_prep_centroids, dim3((P.kp * P.DP + 255) / 256), dim3(256), 0, s, C, k, d,
                       P.kp, P.DP, parts);
    hipLaunchKernelGGL(k_centroid_norms, dim3(P.kp), dim3(64), 0, s, C, k, d, P.kp, cn);
    const unsigned blocks = static_cast<unsigned>(P.blocks);
#define CSC_MF_F(TF, DPV, TV, FV)                                                                   \
  hipLaunchKernelGGL((k_assign_mf<TF, DPV, TV, (TV == 2 ? 8 : 4), FV>), dim3(blocks), dim3(64 * P.wv), \
                     P.lds, s,                                                                    \
                     static_cast<const TF*>(F), ldf, n, d, parts, cn, C, k, P.kp, P.kc, labels,   \
                     best_d2, obj_part)
    // whole 16-byte pieces: the unmasked row loads
    const bool full = d % 8 == 0;
#define CSC_MF(TF, DPV, TV)                  \
  if (full) {                                \
    CSC_MF_F(TF, DPV, TV, true);             \
  } else {                                   \
    CSC_MF_F(TF, DPV, TV, false);            \
  }
#define CSC_MF_DP(TF, TV)                    \
  switch (P.DP) {                            \
    case 32: CSC_MF(TF, 32, TV); break;      \
    case 64: CSC_MF(TF, 64, TV); break;      \
    case 128: CSC_MF(TF, 128, TV); break;    \
    default: CSC_MF(TF, 256, TV); break;     \
  }
    if (f_dt == CSC_F32) { CSC_MF_DP(float, 1) }
    else if (P.T == 1) { CSC_MF_DP(uint16_t, 1) }
    else { CSC_MF_DP(uint16_t, 2) }
#undef CSC_MF_DP
#undef CSC_MF
#undef CSC_MF_F
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
                                float* sums, int32_t* counts, void* work, size_t work_bytes,
                                hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  if (!C || !labels) return fail(CSC_E_ARG, "null centroids or labels");
  const KmLayout L = km_layout(n, d, k);
  if (!work || work_bytes < L.total) return fail(CSC_E_ARG, "k-means workspace too small");
  auto* Cp = reinterpret_cast<float*>(static_cast<char*>(work) + L.off_cp);
  CSC_TRY(assign_impl(F, f_dt, ldf, n, d, C, k, labels, best_d2, nullptr, Cp, s));
  // the Lloyd partial sums of the new assignment: the update's fixed-point accumulation
  // (a second pass over F), without the division by the counts
  if (sums || counts) CSC_TRY(update_impl(F, f_dt, ldf, n, d, labels, k, nullptr, counts, work, false, s, sums));
  return CSC_OK;
}

// ---- the assignment without workspace: split centroids in a static device array -------
//
// For callers that cannot allocate (graph capture, serving loops).  The array holds the
// split centroids of the matrix-core path (or the padded ones of the vector path) for
// k <= 240 and d <= 256; each device has its own copy, whose address is looked up once per
// device with that device current.  Every call on a device uses that device's copy, so
// calls that overlap on one device race.

namespace {
constexpr size_t kStaticScratch = 256 * 1024;
__device__ __align__(256) unsigned char scratch[kStaticScratch];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};
}  // namespace

size_t kmeans_static_scratch_bytes() { return kStaticScratch; }

csc_status launch_kmeans_assign_static(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n,
                                       int d, const float* C, int k, int32_t* labels,
                                       float* best_d2, hipStream_t s) {
  CSC_TRY(check_f(F, f_dt, ldf, n, d, k));
  if (!C || !labels) return fail(CSC_E_ARG, "null centroids or labels");
  if (k > 240 || d > 256 || assign_scratch_bytes(k, d) > kStaticScratch)
    return fail(CSC_E_ARG, "the allocation-free assignment takes k <= 240 and d <= 256 (its static "
                           "scratch holds " + std::to_string(kStaticScratch) + " bytes)");
  int dev = 0;
  CSC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CSC_E_ARG, "device index out of range");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      CSC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p) return fail(CSC_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
      g_scratch[dev] = p;
    }
    ptr = g_scratch[dev];
  }
  return assign_impl(F, f_dt, ldf, n, d, C, k, labels, best_d2, nullptr, static_cast<float*>(ptr), s);
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
  // the 16-byte path needs aligned rows and whole 16-byte pieces (its loads are unmasked)
  const bool vec = rows_aligned(F, f_dt, ldf) && d % static_cast<int>(16 / dtype_size(f_dt)) == 0;
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
  const int npc = (d + (f32 ? 63 : 127)) / (f32 ? 64 : 128);  // 16-byte pieces per lane
#define CSC_PPD_N(TF, V, NP)                                                                       \
  hipLaunchKernelGGL((k_pp_dist<TF, V, NP>), dim3(static_cast<unsigned>(nblk)), dim3(kThreads), 0, \
                     s, static_cast<const TF*>(F), ldf, n, d, dp, C, j - 1, first, cd, own, d2, bsum)
#define CSC_PPD(TF, V)                               \
  switch (npc) {                                     \
    case 1: CSC_PPD_N(TF, V, 1); break;              \
    case 2: CSC_PPD_N(TF, V, 2); break;              \
    case 3: CSC_PPD_N(TF, V, 3); break;              \
    default: CSC_PPD_N(TF, V, 4); break;             \
  }
#define CSC_PPD16(V)                                 \
  if (npc == 1) { CSC_PPD_N(uint16_t, V, 1); } else { CSC_PPD_N(uint16_t, V, 2); }
  int32_t* own = reinterpret_cast<int32_t*>(base + L.off_own);
  double* cd = reinterpret_cast<double*>(base + L.off_cd);
  for (int j = 1; j < k; ++j) {
    const int first = j == 1 ? 1 : 0;
    if (!first) hipLaunchKernelGGL(k_pp_cdist, dim3(j - 1), dim3(64), 0, s, C, d, j - 1, cd);
    if (f32) {
      if (vec) { CSC_PPD(float, true) } else { CSC_PPD(float, false) }
      hipLaunchKernelGGL(k_pp_pick<float>, dim3(1), dim3(1024), 0, s, static_cast<const float*>(F), ldf,
                         n, d, d2, bsum, nblk, rows_per_blk, u, j, C, idx, sel);
    } else {
      if (vec) { CSC_PPD16(true) } else { CSC_PPD16(false) }
      hipLaunchKernelGGL(k_pp_pick<uint16_t>, dim3(1), dim3(1024), 0, s,
                         static_cast<const uint16_t*>(F), ldf, n, d, d2, bsum, nblk, rows_per_blk, u,
                         j, C, idx, sel);
    }
  }
#undef CSC_PPD
#undef CSC_PPD16
#undef CSC_PPD_N
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
  hipLaunchKernelGGL(k_upd_clear, dim3(1), dim3(256), 0, s, static_cast<int32_t*>(nullptr), 0, mx);
  CSC_TRY(launch_maxabs(F, f_dt, ldf, n, d, mx, s));
  const int64_t nparts = assign_parts(n, d, k, F, f_dt, ldf);
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
