// Fixed-order FP64 dot products and the Philox4x32-10 Gaussian / uniform draws.
#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kThreads = 256;
constexpr int64_t kDotBlocks = 2048;

__device__ inline double load_d(const void* p, int dt, int64_t i) {
  if (dt == CSC_F32) return static_cast<double>(static_cast<const float*>(p)[i]);
  if (dt == CSC_BF16) return static_cast<double>(bf16_to_f32(static_cast<const uint16_t*>(p)[i]));
  return static_cast<const double*>(p)[i];
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
  return s;
}

__global__ void k_dot_part(const void* X, int x_dt, int64_t ldx, const void* Y, int y_dt,
                           int64_t ldy, int64_t n, int w, double* part) {
  const int64_t total = n * w;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  double s = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < total;
       i += stride) {
    const int64_t r = i / w;
    const int64_t c = i - r * w;
    s += load_d(X, x_dt, r * ldx + c) * load_d(Y, y_dt, r * ldy + c);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_dot_final(const double* part, int nb, double* out) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) s += part[b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
struct Ctr { uint32_t c[4]; };

__device__ inline Ctr philox10(Ctr x, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * x.c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, x.c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * x.c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x.c[2]);
    Ctr y;
    y.c[0] = hi1 ^ x.c[1] ^ k0;
    y.c[1] = lo1;
    y.c[2] = hi0 ^ x.c[3] ^ k1;
    y.c[3] = lo0;
    x = y;
  }
  return x;
}

__device__ inline double u53(uint32_t lo, uint32_t hi) {
  const uint64_t v = (static_cast<uint64_t>(hi) << 32) | lo;
  return static_cast<double>(v >> 11) * 0x1.0p-53 + 0x1.0p-54;
}

__device__ inline void store_elem(void* X, int dt, int64_t i, double v) {
  if (dt == CSC_F32) static_cast<float*>(X)[i] = static_cast<float>(v);
  else if (dt == CSC_BF16) static_cast<uint16_t*>(X)[i] = f32_to_bf16(static_cast<float>(v));
  else static_cast<double*>(X)[i] = v;
}

__global__ void k_randn(void* X, int dt, int64_t n, int w, int64_t ldx, int64_t row0,
                        uint32_t s_lo, uint32_t s_hi, uint32_t t_lo, uint32_t t_hi, double sigma) {
  const int npair = (w + 1) / 2;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * npair) return;
  const int64_t r = idx / npair;
  const int q = static_cast<int>(idx - r * npair);
  Ctr c;
  c.c[0] = static_cast<uint32_t>(r + row0);
  c.c[1] = static_cast<uint32_t>(q);
  c.c[2] = t_lo;
  c.c[3] = t_hi;
  const Ctr o = philox10(c, s_lo, s_hi);
  const double u1 = u53(o.c[0], o.c[1]);
  const double u2 = u53(o.c[2], o.c[3]);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  const int64_t base = r * ldx + 2 * q;
  store_elem(X, dt, base, sigma * rad * cos(ang));
  if (2 * q + 1 < w) store_elem(X, dt, base + 1, sigma * rad * sin(ang));
}

__global__ void k_uniforms(double* u, int count, uint32_t s_lo, uint32_t s_hi, uint32_t t_lo,
                           uint32_t t_hi) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  Ctr c;
  c.c[0] = static_cast<uint32_t>(j);
  c.c[1] = 0;
  c.c[2] = t_lo;
  c.c[3] = t_hi;
  const Ctr o = philox10(c, s_lo, s_hi);
  u[j] = u53(o.c[0], o.c[1]);
}

}  // namespace

size_t dot_workspace(int64_t) { return align_up(kDotBlocks * sizeof(double)); }

csc_status launch_dot(const void* X, csc_dtype x_dt, int64_t ldx, const void* Y, csc_dtype y_dt,
                      int64_t ldy, int64_t n, int w, double* result, void* work,
                      size_t work_bytes, hipStream_t s) {
  if (work_bytes < dot_workspace(n) || !work) return fail(CSC_E_ARG, "dot workspace too small");
  if (n < 0 || w < 1 || ldx < w || ldy < w) return fail(CSC_E_ARG, "bad dot sizes");
  const int64_t total = n * w;
  int nb = static_cast<int>(std::min<int64_t>(kDotBlocks, (total + kThreads - 1) / kThreads));
  if (nb < 1) nb = 1;
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(kThreads), 0, s, X, int(x_dt), ldx, Y, int(y_dt),
                     ldy, n, w, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kThreads), 0, s, part, nb, result);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status launch_randn(void* X, csc_dtype dt, int64_t n, int w, int64_t ldx, int64_t row0,
                        uint64_t seed, uint64_t stream_id, double sigma, hipStream_t s) {
  if (!X || n < 0 || w < 1 || ldx < w) return fail(CSC_E_ARG, "bad randn arguments");
  if (row0 < 0 || n + row0 > (int64_t(1) << 32)) return fail(CSC_E_ARG, "row index exceeds 32 bits");
  const int64_t total = n * ((w + 1) / 2);
  if (total == 0) return CSC_OK;
  hipLaunchKernelGGL(k_randn, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s,
                     X, int(dt), n, w, ldx, row0, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32), static_cast<uint32_t>(stream_id),
                     static_cast<uint32_t>(stream_id >> 32), sigma);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

csc_status launch_uniforms(double* u, int count, uint64_t seed, uint64_t stream_id,
                           hipStream_t s) {
  if (!u || count < 0) return fail(CSC_E_ARG, "bad uniforms arguments");
  if (count == 0) return CSC_OK;
  hipLaunchKernelGGL(k_uniforms, dim3((count + 255) / 256), dim3(256), 0, s, u, count,
                     static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32),
                     static_cast<uint32_t>(stream_id), static_cast<uint32_t>(stream_id >> 32));
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace csc
