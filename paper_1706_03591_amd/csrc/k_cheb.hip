// Fused Chebyshev recurrence step (Sec. 2.2, Step 1; Sec. 3.2).
//
// One launch computes, for every row r of one column tile,
//     acc      = sum_{c in row r} A_rc Z_j[c, :]                       (sparse gather)
//     Z_{j+1}  = 2 (alpha Z_j[r] - beta acc) - Z_{j-1}[r]               (three-term step)
//     Y[r]    += a_{j+1} Z_{j+1}[r]                                     (coefficient accumulate)
// with L~ = alpha I - beta A (alpha = 2 / lmax - 1, beta = 2 / lmax) for the normalized
// Laplacian; for the combinatorial one A is W and alpha becomes the per-row
// 2 d_r / lmax - 1 (L~ = (2 / lmax)(D - W) - I).  Z_{j+1} overwrites
// Z_{j-1} in place: row r reads its own Z_{j-1} row before writing it and no other row
// reads Z_{j-1}.  Optionally the per-row dot products <Z_j, Z_j> and <Z_{j+1}, Z_j> are
// reduced (FP64, fixed order) for the doubled Chebyshev moments.
//
// Layout.  Iterates live in the workspace as column tiles: tile t is a contiguous n x wt
// array (row-major), so a gathered row segment is wt * sizeof(T) contiguous bytes and the
// tile that the whole grid gathers from is as small as the cache it should stay in.  Blocks
// are numbered tile-major, so the blocks in flight at any time work on one tile.  A block
// stages its rows' column indices and values in LDS with one coalesced pass; each row is
// served by `LPR` lanes that each own 16 bytes of the row (4 FP32 or 8 BF16 columns), so a
// gather is one 16-byte load per lane and one contiguous segment per row group.
//
// Iterate modes: FP32; BF16 or F16 (iterates rounded to BF16 / IEEE binary16 at every step);
// BF16S or F16S (16-bit copies of the iterates for the gathers and the kept basis, while the
// recurrence state Z_{j-1}, Z_j, Z_{j+1} of each row stays in a separate FP32 tiled array
// with the same element offsets).
#include <type_traits>

#include "csc_internal.h"

namespace csc {

namespace {

constexpr int kThreads = 256;
constexpr int kStageCap = 2048;  // CSR entries staged in LDS per block
constexpr int kLight = 32;       // a heavy block's rows up to this many entries: one row group

enum : int { F_FIRST = 1, F_ACC = 2, F_LAST = 4, F_MOM = 8, F_STORE = 16, F_OWN = 32 };

// Tag types of the split iterate modes (16-bit gathered copies, FP32 state).  The 16-bit
// storage types are uint16_t (BF16 bits) and _Float16 (IEEE binary16).
struct Bf16S {};
struct F16S {};
template <typename TZ>
constexpr bool kSplit = std::is_same<TZ, Bf16S>::value || std::is_same<TZ, F16S>::value;
template <typename TZ>
using GatherT = typename std::conditional<
    std::is_same<TZ, Bf16S>::value, uint16_t,
    typename std::conditional<std::is_same<TZ, F16S>::value, _Float16, TZ>::type>::type;

// Conversions of a 16-bit storage type: to(f) rounds to nearest even and returns the bits,
// from(bits) widens exactly.
template <typename T16>
struct Cvt16;
template <>
struct Cvt16<uint16_t> {
  __device__ static inline uint16_t to(float f) { return f32_to_bf16(f); }
  __device__ static inline float from(uint16_t h) { return bf16_to_f32(h); }
};
template <>
struct Cvt16<_Float16> {
  __device__ static inline uint16_t to(float f) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(f));
  }
  __device__ static inline float from(uint16_t h) {
    return static_cast<float>(__builtin_bit_cast(_Float16, h));
  }
};

template <typename TZ>
struct Pack;

template <>
struct Pack<float> {
  static constexpr int VEC = 4;
  __device__ static inline void unpack(const uint4& u, float* f) {
    f[0] = __uint_as_float(u.x);
    f[1] = __uint_as_float(u.y);
    f[2] = __uint_as_float(u.z);
    f[3] = __uint_as_float(u.w);
  }
  // round to storage (identity) and return the stored values
  __device__ static inline uint4 pack(float* f) {
    return make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                      __float_as_uint(f[3]));
  }
};

// eight 16-bit values per 16 bytes, element 2i in the low half of word i
template <typename T16>
struct Pack16 {
  static constexpr int VEC = 8;
  __device__ static inline void unpack(const uint4& u, float* f) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[2 * i] = Cvt16<T16>::from(static_cast<uint16_t>(w[i] & 0xffffu));
      f[2 * i + 1] = Cvt16<T16>::from(static_cast<uint16_t>(w[i] >> 16));
    }
  }
  // round to storage and return the stored values in f
  __device__ static inline uint4 pack(float* f) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint16_t lo = Cvt16<T16>::to(f[2 * i]);
      const uint16_t hi = Cvt16<T16>::to(f[2 * i + 1]);
      f[2 * i] = Cvt16<T16>::from(lo);
      f[2 * i + 1] = Cvt16<T16>::from(hi);
      w[i] = static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
};
template <>
struct Pack<uint16_t> : Pack16<uint16_t> {};
template <>
struct Pack<_Float16> : Pack16<_Float16> {};

template <typename TV>
__device__ inline float val_f(TV v);
template <>
__device__ inline float val_f<float>(float v) { return v; }
template <>
__device__ inline float val_f<uint16_t>(uint16_t v) { return bf16_to_f32(v); }

__device__ inline uint4 ld16(const void* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ inline void st16(void* p, const uint4& v) { *reinterpret_cast<uint4*>(p) = v; }

// eight FP32 state values (32 bytes) of one lane
__device__ inline void ld8f(const float* p, float* f) {
  const uint4 a = ld16(p), b = ld16(p + 4);
  f[0] = __uint_as_float(a.x); f[1] = __uint_as_float(a.y);
  f[2] = __uint_as_float(a.z); f[3] = __uint_as_float(a.w);
  f[4] = __uint_as_float(b.x); f[5] = __uint_as_float(b.y);
  f[6] = __uint_as_float(b.z); f[7] = __uint_as_float(b.w);
}
__device__ inline void st8f(float* p, const float* f) {
  st16(p, make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                     __float_as_uint(f[3])));
  st16(p + 4, make_uint4(__float_as_uint(f[4]), __float_as_uint(f[5]), __float_as_uint(f[6]),
                         __float_as_uint(f[7])));
}

struct StepParams {
  const int32_t* rowptr;
  const int32_t* colidx;
  const void* vals;
  const void* zcur;
  const void* zprev;
  void* zout;
  const float* scur;   // BF16S: FP32 state Z_j (tiled like the copies)
  const float* sprev;  // BF16S: FP32 state Z_{j-1}
  float* sout;         // BF16S: FP32 state Z_{j+1} (in place over Z_{j-1})
  float* acc;      // row-major n x wpad
  int64_t ld_acc;  // = wpad
  void* yout;      // final output (row-major, ldy, y_dt) on the last step, else null
  int64_t ldy;
  int y_dt;
  int w;
  int64_t n;
  int64_t row_blocks;
  float alpha, beta, coef;
  const double* coef_dev;  // device FP64 coefficient; when set it replaces `coef` (graph replay
                           // with coefficients that change between replays)
  float gam;           // combinatorial: own-row factor alpha + gam d_r
  const float* diag;   // combinatorial: d_r; null for the normalized Laplacian
  int flags;
  double* mom_part;  // [2][gridDim.x]
};

// L~ = (2 / lmax) L - I written as diag(alpha + gam d) - beta S, with S the stored matrix:
// normalized (S = A): alpha = 2 / lmax - 1, gam = 0; combinatorial (S = W): alpha = -1,
// gam = beta = 2 / lmax.
struct OpScale {
  float alpha, beta, gam;
  const float* diag;
  bool own() const { return alpha != 0.f || diag != nullptr; }
};
inline OpScale op_scale(const Graph* g, double lmax) {
  const float b = static_cast<float>(2.0 / lmax);
  if (g->lap == CSC_LAP_COMBINATORIAL) return {-1.f, b, b, g->diag};
  return {static_cast<float>(2.0 / lmax - 1.0), b, 0.f, nullptr};
}
inline void set_op(StepParams& p, const OpScale& o) {
  p.alpha = o.alpha;
  p.beta = o.beta;
  p.gam = o.gam;
  p.diag = o.diag;
}

__device__ inline void store_out(void* y, int dt, int64_t idx, float v) {
  if (dt == CSC_F32) static_cast<float*>(y)[idx] = v;
  else if (dt == CSC_BF16) static_cast<uint16_t*>(y)[idx] = f32_to_bf16(v);
  else static_cast<double*>(y)[idx] = static_cast<double>(v);
}

// Fixed-order block reduction of two doubles; result valid in thread 0.
__device__ inline void block_reduce2(double& a, double& b) {
  __shared__ double red[2][kThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63;
  if (lid == 0) { red[0][wid] = a; red[1][wid] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0; b = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) { a += red[0][i]; b += red[1][i]; }
  }
}

// Body of one step for block `bid` of a launch of `nblocks` blocks (the batched launch runs
// several snapshots' steps, each with its own parameters and block range).
template <typename TZ, typename TV, int LPR>
__device__ inline void step_body(const StepParams& p, const int64_t bid, const int64_t nblocks) {
  constexpr bool MIX = kSplit<TZ>;
  using TG = GatherT<TZ>;
  using P = Pack<TG>;
  constexpr int VEC = P::VEC;
  constexpr int WT = LPR * VEC;
  constexpr int RPB = kThreads / LPR;
  __shared__ int32_t s_col[kStageCap];
  __shared__ float s_val[kStageCap];

  const int64_t tile = bid / p.row_blocks;
  const int64_t rb = bid - tile * p.row_blocks;
  const int64_t r0 = rb * RPB;
  const int64_t r1 = min(r0 + RPB, p.n);
  const int32_t e0 = p.rowptr[r0];
  const int32_t e1 = p.rowptr[r1];
  const int32_t cnt = e1 - e0;
  const bool staged = cnt <= kStageCap;
  const TV* vals = static_cast<const TV*>(p.vals);
  if (staged) {
    for (int32_t i = threadIdx.x; i < cnt; i += kThreads) {
      s_col[i] = p.colidx[e0 + i];
      s_val[i] = val_f<TV>(vals[e0 + i]);
    }
  }
  __syncthreads();

  const int64_t row = r0 + threadIdx.x / LPR;
  const int grp = threadIdx.x / LPR;
  const int lane = threadIdx.x % LPR;
  const int64_t tile_off = tile * p.n * WT;  // elements
  const TG* zc = static_cast<const TG*>(p.zcur) + tile_off + lane * VEC;
  double d1 = 0.0, d2 = 0.0;

  float acc[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) acc[i] = 0.f;
  if (staged) {
    if (row < p.n) {
      const int32_t rs = p.rowptr[row], re = p.rowptr[row + 1];
      int32_t e = rs;
      for (; e + 8 <= re; e += 8) {
        const int32_t l = e - e0;
        uint4 g[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) g[q] = ld16(zc + static_cast<int64_t>(s_col[l + q]) * WT);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float f[VEC];
          P::unpack(g[q], f);
          const float v = s_val[l + q];
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v, f[i], acc[i]);
        }
      }
      for (; e + 4 <= re; e += 4) {
        const int32_t l = e - e0;
        const int32_t c0 = s_col[l], c1 = s_col[l + 1], c2 = s_col[l + 2], c3 = s_col[l + 3];
        const float v0 = s_val[l], v1 = s_val[l + 1], v2 = s_val[l + 2], v3 = s_val[l + 3];
        const uint4 g0 = ld16(zc + static_cast<int64_t>(c0) * WT);
        const uint4 g1 = ld16(zc + static_cast<int64_t>(c1) * WT);
        const uint4 g2 = ld16(zc + static_cast<int64_t>(c2) * WT);
        const uint4 g3 = ld16(zc + static_cast<int64_t>(c3) * WT);
        float f[VEC];
        P::unpack(g0, f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v0, f[i], acc[i]);
        P::unpack(g1, f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v1, f[i], acc[i]);
        P::unpack(g2, f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v2, f[i], acc[i]);
        P::unpack(g3, f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v3, f[i], acc[i]);
      }
      for (; e < re; ++e) {
        const int32_t l = e - e0;
        const uint4 g = ld16(zc + static_cast<int64_t>(s_col[l]) * WT);
        float f[VEC];
        P::unpack(g, f);
        const float v = s_val[l];
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v, f[i], acc[i]);
      }
    }
  } else {
    // Heavy block (more CSR entries than the LDS stage holds, e.g. the hubs of a power-law
    // graph).  Its light rows (at most kLight entries) are summed by their own row group,
    // reading the CSR from global memory.  Its other rows are taken one at a time by all RPB
    // row groups: the row's entries pass through LDS in chunks of kChunk (a multiple of RPB),
    // group g sums the entries rs + g, rs + g + RPB, ... eight gathers at a time, and the
    // partial sums meet in LDS in group order, so the result does not depend on scheduling.
    constexpr int kChunk = kStageCap / 2;
    static_assert(kThreads * VEC <= kStageCap, "reduction buffer must fit the stage");
    static_assert(kChunk % RPB == 0, "chunks must keep each group's entries");
    // reduction buffer: the upper halves of the stage (kThreads * VEC floats)
    auto red = [&](int i) -> float& {
      return i < kStageCap / 2 ? reinterpret_cast<float*>(s_col)[kStageCap / 2 + i] : s_val[i];
    };
    if (row < p.n) {
      const int32_t rs = p.rowptr[row], re = p.rowptr[row + 1];
      if (re - rs <= kLight) {
        int32_t e = rs;
        for (; e + 8 <= re; e += 8) {
          int32_t c[8];
          float v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) { c[q] = p.colidx[e + q]; v[q] = val_f<TV>(vals[e + q]); }
          uint4 g[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) g[q] = ld16(zc + static_cast<int64_t>(c[q]) * WT);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float f[VEC];
            P::unpack(g[q], f);
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v[q], f[i], acc[i]);
          }
        }
        for (; e < re; ++e) {
          const uint4 g = ld16(zc + static_cast<int64_t>(p.colidx[e]) * WT);
          float f[VEC];
          P::unpack(g, f);
          const float v = val_f<TV>(vals[e]);
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] = fmaf(v, f[i], acc[i]);
        }
      }
    }
    for (int rr = 0; rr < RPB && r0 + rr < p.n; ++rr) {
      const int64_t rw = r0 + rr;
      const int32_t rs = p.rowptr[rw], re = p.rowptr[rw + 1];
      if (re - rs <= kLight) continue;  // (uniform over the block)
      float part[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) part[i] = 0.f;
      for (int32_t c0 = rs; c0 < re; c0 += kChunk) {
        const int32_t cn = min(kChunk, re - c0);
        __syncthreads();  // the previous chunk's readers are done
        for (int32_t i = threadIdx.x; i < cn; i += kThreads) {
          s_col[i] = p.colidx[c0 + i];
          s_val[i] = val_f<TV>(vals[c0 + i]);
        }
        __syncthreads();
        int32_t l = grp;
        for (; l + 7 * RPB < cn; l += 8 * RPB) {
          uint4 g[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) g[q] = ld16(zc + static_cast<int64_t>(s_col[l + q * RPB]) * WT);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float f[VEC];
            P::unpack(g[q], f);
            const float v = s_val[l + q * RPB];
#pragma unroll
            for (int i = 0; i < VEC; ++i) part[i] = fmaf(v, f[i], part[i]);
          }
        }
        for (; l < cn; l += RPB) {
          const uint4 g = ld16(zc + static_cast<int64_t>(s_col[l]) * WT);
          float f[VEC];
          P::unpack(g, f);
          const float v = s_val[l];
#pragma unroll
          for (int i = 0; i < VEC; ++i) part[i] = fmaf(v, f[i], part[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < VEC; ++i) red((grp * LPR + lane) * VEC + i) = part[i];
      __syncthreads();
      if (grp == rr) {
        for (int g = 0; g < RPB; ++g)
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] += red((g * LPR + lane) * VEC + i);
      }
      __syncthreads();
    }
  }

  if (row < p.n) {
    const int64_t own = row * WT;  // element offset of this row within the tile
    const int64_t eoff = tile_off + lane * VEC + own;
    float zj[VEC];
    if (p.flags & F_OWN) {
      if constexpr (MIX) ld8f(p.scur + eoff, zj);
      else P::unpack(ld16(zc + own), zj);
    } else {
#pragma unroll
      for (int i = 0; i < VEC; ++i) zj[i] = 0.f;
    }
    const float al = p.diag ? fmaf(p.gam, p.diag[row], p.alpha) : p.alpha;
    float zn[VEC];
    if (p.flags & F_FIRST) {
#pragma unroll
      for (int i = 0; i < VEC; ++i) zn[i] = fmaf(al, zj[i], -p.beta * acc[i]);
    } else {
      float zp[VEC];
      if constexpr (MIX) ld8f(p.sprev + eoff, zp);
      else P::unpack(ld16(static_cast<const TG*>(p.zprev) + eoff), zp);
#pragma unroll
      for (int i = 0; i < VEC; ++i)
        zn[i] = 2.f * fmaf(al, zj[i], -p.beta * acc[i]) - zp[i];
    }
    if constexpr (MIX) {
      // the state keeps FP32; only the gathered copy is rounded
      if (p.flags & F_STORE) {
        st8f(p.sout + eoff, zn);
        float cp[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) cp[i] = zn[i];
        st16(static_cast<TG*>(p.zout) + eoff, P::pack(cp));
      }
    } else {
      const uint4 packed = P::pack(zn);  // zn now holds the stored (rounded) values
      if (p.flags & F_STORE) st16(static_cast<TG*>(p.zout) + eoff, packed);
    }
    if (p.flags & F_MOM) {
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        s1 = fmaf(zj[i], zj[i], s1);
        s2 = fmaf(zn[i], zj[i], s2);
      }
      d1 = s1;
      d2 = s2;
    }
    if (p.flags & F_ACC) {
      const int64_t col0 = tile * WT + lane * VEC;
      float* ap = p.acc + row * p.ld_acc + col0;
      const float cf = p.coef_dev ? static_cast<float>(*p.coef_dev) : p.coef;
      float y[VEC];
#pragma unroll
      for (int i = 0; i < VEC; i += 4) {
        float4 t4 = *reinterpret_cast<const float4*>(ap + i);
        y[i] = fmaf(cf, zn[i], t4.x);
        y[i + 1] = fmaf(cf, zn[i + 1], t4.y);
        y[i + 2] = fmaf(cf, zn[i + 2], t4.z);
        y[i + 3] = fmaf(cf, zn[i + 3], t4.w);
      }
      if (p.yout) {
#pragma unroll
        for (int i = 0; i < VEC; ++i)
          if (col0 + i < p.w) store_out(p.yout, p.y_dt, row * p.ldy + col0 + i, y[i]);
      } else {
#pragma unroll
        for (int i = 0; i < VEC; i += 4)
          *reinterpret_cast<float4*>(ap + i) = make_float4(y[i], y[i + 1], y[i + 2], y[i + 3]);
      }
    }
  }
  if (p.flags & F_MOM) {
    block_reduce2(d1, d2);
    if (threadIdx.x == 0) {
      p.mom_part[bid] = d1;
      p.mom_part[nblocks + bid] = d2;
    }
  }
}

template <typename TZ, typename TV, int LPR>
__global__ __launch_bounds__(kThreads) void k_step(StepParams p) {
  step_body<TZ, TV, LPR>(p, blockIdx.x, gridDim.x);
}

// Several independent steps (one per snapshot of a batch, same n and tile shape) in one
// launch: block b runs step b / per of the batch.
constexpr int kMaxBatch = 8;
struct StepBatch {
  StepParams p[kMaxBatch];
  int64_t per;
};

template <typename TZ, typename TV, int LPR>
__global__ __launch_bounds__(kThreads) void k_step_batch(StepBatch b) {
  const int s = static_cast<int>(blockIdx.x / b.per);
  step_body<TZ, TV, LPR>(b.p[s], blockIdx.x - s * b.per, b.per);
}

// Z_0 (tiled, iter type) from X (row-major, x_dt); acc = a0 * Z_0 when acc != null.
template <typename TZ>
__global__ void k_init(const void* X, int x_dt, int64_t ldx, int64_t n, int w, int wpad, int wt,
                       TZ* z0, float* acc, float a0, float* s0, const double* a0_dev) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * wpad) return;
  if (a0_dev) a0 = static_cast<float>(*a0_dev);
  const int64_t row = idx / wpad;
  const int col = static_cast<int>(idx - row * wpad);
  float x = 0.f;
  if (col < w) {
    const int64_t src = row * ldx + col;
    if (x_dt == CSC_F32) x = static_cast<const float*>(X)[src];
    else if (x_dt == CSC_BF16) x = bf16_to_f32(static_cast<const uint16_t*>(X)[src]);
    else x = static_cast<float>(static_cast<const double*>(X)[src]);
  }
  const int tile = col / wt, c = col - tile * wt;
  const int64_t e = static_cast<int64_t>(tile) * n * wt + row * wt + c;
  float stored;
  if constexpr (sizeof(TZ) == 4) {
    stored = x;
    z0[e] = stored;
  } else {
    const uint16_t h = Cvt16<TZ>::to(x);
    reinterpret_cast<uint16_t*>(z0)[e] = h;
    stored = s0 ? x : Cvt16<TZ>::from(h);  // split modes: the state keeps the FP32 value
    if (s0) s0[e] = x;
  }
  if (acc) acc[row * wpad + col] = a0 * stored;
}

// k_init for eight columns per thread (16-byte loads and stores): X is F32 or BF16 with
// 16-byte aligned rows and w a multiple of 8, so a group of eight columns lies wholly inside
// or wholly past w, and inside one tile (wt is a multiple of 8).  Same values as k_init.
template <typename TZ>
__global__ void k_init8(const void* X, int x_dt, int64_t ldx, int64_t n, int w, int wpad, int wt,
                        TZ* z0, float* acc, float a0, float* s0, const double* a0_dev) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int gpr = wpad / 8;
  if (g >= n * gpr) return;
  if (a0_dev) a0 = static_cast<float>(*a0_dev);
  const int64_t row = g / gpr;
  const int col = static_cast<int>(g - row * gpr) * 8;
  float x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = 0.f;
  if (col < w) {
    if (x_dt == CSC_BF16) {
      const uint4 u = ld16(static_cast<const uint16_t*>(X) + row * ldx + col);
      const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) {
        x[2 * k2] = __uint_as_float(wd[k2] << 16);
        x[2 * k2 + 1] = __uint_as_float(wd[k2] & 0xffff0000u);
      }
    } else {
      const float* xp = static_cast<const float*>(X) + row * ldx + col;
      const uint4 u0 = ld16(xp), u1 = ld16(xp + 4);
      x[0] = __uint_as_float(u0.x); x[1] = __uint_as_float(u0.y);
      x[2] = __uint_as_float(u0.z); x[3] = __uint_as_float(u0.w);
      x[4] = __uint_as_float(u1.x); x[5] = __uint_as_float(u1.y);
      x[6] = __uint_as_float(u1.z); x[7] = __uint_as_float(u1.w);
    }
  }
  const int tile = col / wt, c = col - tile * wt;
  const int64_t e = static_cast<int64_t>(tile) * n * wt + row * wt + c;
  float stored[8];
  if constexpr (sizeof(TZ) == 4) {
#pragma unroll
    for (int i = 0; i < 8; ++i) stored[i] = x[i];
    st8f(reinterpret_cast<float*>(z0) + e, x);
  } else {
    uint32_t wd[4];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      const uint16_t lo = Cvt16<TZ>::to(x[2 * k2]), hi = Cvt16<TZ>::to(x[2 * k2 + 1]);
      wd[k2] = static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 16);
      stored[2 * k2] = s0 ? x[2 * k2] : Cvt16<TZ>::from(lo);  // split modes keep FP32
      stored[2 * k2 + 1] = s0 ? x[2 * k2 + 1] : Cvt16<TZ>::from(hi);
    }
    st16(z0 + e, make_uint4(wd[0], wd[1], wd[2], wd[3]));
    if (s0) st8f(s0 + e, x);
  }
  if (acc) {
    float av[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) av[i] = a0 * stored[i];
    st8f(acc + row * wpad + col, av);
  }
}

__global__ void k_acc_out(const float* acc, int64_t n, int w, int wpad, void* y, int y_dt,
                          int64_t ldy) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * w) return;
  const int64_t row = idx / w;
  const int col = static_cast<int>(idx - row * w);
  store_out(y, y_dt, row * ldy + col, acc[row * wpad + col]);
}

// sums[q] = sum_b part[q * nb + b] in a fixed order (one block per q).
__global__ void k_reduce_rows(const double* part, int64_t nb, double* sums) {
  const int q = blockIdx.x;
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kThreads) s += part[q * nb + b];
  double dummy = 0.0;
  block_reduce2(s, dummy);
  if (threadIdx.x == 0) sums[q] = s;
}

// Doubling: mu_0 = d1(0), mu_1 = d2(0), mu_2j = 2 d1(j) - mu_0, mu_2j+1 = 2 d2(j) - mu_1.
__global__ void k_moments(const double* sums, int J, int m, double* mu) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double mu0 = sums[0], mu1 = sums[1];
  mu[0] = mu0;
  if (m >= 1) mu[1] = mu1;
  for (int j = 1; j <= J; ++j) {
    if (2 * j <= m) mu[2 * j] = 2.0 * sums[2 * j] - mu0;
    if (2 * j + 1 <= m) mu[2 * j + 1] = 2.0 * sums[2 * j + 1] - mu1;
  }
}

using StepFn = void (*)(StepParams);

template <typename TZ>
StepFn pick_step(int lpr, csc_dtype val_dt) {
  const bool vb = val_dt == CSC_BF16;
  switch (lpr) {
    case 4: return vb ? k_step<TZ, uint16_t, 4> : k_step<TZ, float, 4>;
    case 8: return vb ? k_step<TZ, uint16_t, 8> : k_step<TZ, float, 8>;
    case 16: return vb ? k_step<TZ, uint16_t, 16> : k_step<TZ, float, 16>;
    default: return vb ? k_step<TZ, uint16_t, 32> : k_step<TZ, float, 32>;
  }
}

const int kLpr[] = {4, 8, 16, 32};

using BatchFn = void (*)(StepBatch);

template <typename TZ>
BatchFn pick_batch(int lpr, csc_dtype val_dt) {
  const bool vb = val_dt == CSC_BF16;
  switch (lpr) {
    case 4: return vb ? k_step_batch<TZ, uint16_t, 4> : k_step_batch<TZ, float, 4>;
    case 8: return vb ? k_step_batch<TZ, uint16_t, 8> : k_step_batch<TZ, float, 8>;
    case 16: return vb ? k_step_batch<TZ, uint16_t, 16> : k_step_batch<TZ, float, 16>;
    default: return vb ? k_step_batch<TZ, uint16_t, 32> : k_step_batch<TZ, float, 32>;
  }
}

StepFn step_fn(csc_dtype iter_dt, int lpr, csc_dtype val_dt) {
  switch (iter_dt) {
    case CSC_F32: return pick_step<float>(lpr, val_dt);
    case CSC_BF16S: return pick_step<Bf16S>(lpr, val_dt);
    case CSC_F16: return pick_step<_Float16>(lpr, val_dt);
    case CSC_F16S: return pick_step<F16S>(lpr, val_dt);
    default: return pick_step<uint16_t>(lpr, val_dt);
  }
}

BatchFn batch_fn(csc_dtype iter_dt, int lpr, csc_dtype val_dt) {
  switch (iter_dt) {
    case CSC_F32: return pick_batch<float>(lpr, val_dt);
    case CSC_BF16S: return pick_batch<Bf16S>(lpr, val_dt);
    case CSC_F16: return pick_batch<_Float16>(lpr, val_dt);
    case CSC_F16S: return pick_batch<F16S>(lpr, val_dt);
    default: return pick_batch<uint16_t>(lpr, val_dt);
  }
}

// Z_0 of the tiled iterates (and of the FP32 state in BF16S mode) from X; acc = a0 Z_0 when
// acc is given.
void launch_init(csc_dtype iter_dt, const void* X, csc_dtype x_dt, int64_t ldx, int64_t n, int w,
                 int wpad, int wt, void* z0, float* acc, float a0, float* s0, hipStream_t s,
                 const double* a0_dev = nullptr) {
  const size_t xs = dtype_size(x_dt);
  if ((x_dt == CSC_F32 || x_dt == CSC_BF16) && w % 8 == 0 && wpad % 8 == 0 && wt % 8 == 0 &&
      reinterpret_cast<uintptr_t>(X) % 16 == 0 && (static_cast<size_t>(ldx) * xs) % 16 == 0) {
    const int64_t groups = n * (wpad / 8);
    const unsigned gb = static_cast<unsigned>((groups + 255) / 256);
    if (iter_dt == CSC_F32)
      hipLaunchKernelGGL(k_init8<float>, dim3(gb), dim3(256), 0, s, X, int(x_dt), ldx, n, w, wpad,
                         wt, static_cast<float*>(z0), acc, a0, static_cast<float*>(nullptr), a0_dev);
    else if (iter_half(iter_dt))
      hipLaunchKernelGGL(k_init8<_Float16>, dim3(gb), dim3(256), 0, s, X, int(x_dt), ldx, n, w,
                         wpad, wt, static_cast<_Float16*>(z0), acc, a0,
                         iter_split(iter_dt) ? s0 : static_cast<float*>(nullptr), a0_dev);
    else
      hipLaunchKernelGGL(k_init8<uint16_t>, dim3(gb), dim3(256), 0, s, X, int(x_dt), ldx, n, w,
                         wpad, wt, static_cast<uint16_t*>(z0), acc, a0,
                         iter_split(iter_dt) ? s0 : static_cast<float*>(nullptr), a0_dev);
    return;
  }
  const int64_t total = n * wpad;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  if (iter_dt == CSC_F32)
    hipLaunchKernelGGL(k_init<float>, dim3(blocks), dim3(256), 0, s, X, int(x_dt), ldx, n, w, wpad,
                       wt, static_cast<float*>(z0), acc, a0, static_cast<float*>(nullptr), a0_dev);
  else if (iter_half(iter_dt))
    hipLaunchKernelGGL(k_init<_Float16>, dim3(blocks), dim3(256), 0, s, X, int(x_dt), ldx, n, w,
                       wpad, wt, static_cast<_Float16*>(z0), acc, a0,
                       iter_split(iter_dt) ? s0 : static_cast<float*>(nullptr), a0_dev);
  else
    hipLaunchKernelGGL(k_init<uint16_t>, dim3(blocks), dim3(256), 0, s, X, int(x_dt), ldx, n, w,
                       wpad, wt, static_cast<uint16_t*>(z0), acc, a0,
                       iter_split(iter_dt) ? s0 : static_cast<float*>(nullptr), a0_dev);
}

}  // namespace

int num_variants() { return 4; }

StepShape variant_shape(int variant, csc_dtype iter_dt) {
  const int vec = iter_dt == CSC_F32 ? 4 : 8;
  if (variant < 0 || variant >= num_variants()) variant = 2;
  return StepShape{kLpr[variant], vec};
}

int default_variant(const Graph* g, int w, csc_dtype iter_dt) {
  const int v = iter_dt == CSC_F32 ? g->variant_f32 : g->variant_bf16;
  if (v >= 0) return v;
  // widest tile that does not exceed the block width (fewest CSR re-reads)
  const int vec = iter_dt == CSC_F32 ? 4 : 8;
  int best = 0;
  for (int i = 0; i < num_variants(); ++i)
    if (kLpr[i] * vec <= std::max(w, kLpr[0] * vec)) best = i;
  return best;
}

FilterPlan make_plan(int64_t n, int w, csc_dtype iter_dt, int variant, int m_for_moments) {
  FilterPlan pl{};
  pl.n = n;
  pl.w = w;
  pl.variant = variant;
  pl.shape = variant_shape(variant, iter_dt);
  pl.iter_dt = iter_dt;
  const int wt = pl.shape.wt();
  pl.ntiles = (w + wt - 1) / wt;
  pl.wpad = pl.ntiles * wt;
  pl.rows_per_block = kThreads / pl.shape.lpr;
  pl.row_blocks = (n + pl.rows_per_block - 1) / pl.rows_per_block;
  const size_t zbytes = align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt));
  const size_t nb = static_cast<size_t>(pl.row_blocks) * pl.ntiles;
  const int J = m_for_moments >= 1 ? m_for_moments / 2 : 0;
  const size_t sbytes = align_up(static_cast<size_t>(n) * pl.wpad * state_size(iter_dt));
  size_t off = 0;
  pl.off_z0 = off; off += zbytes;
  pl.off_z1 = off; off += zbytes;
  pl.off_s0 = off; off += sbytes;
  pl.off_s1 = off; off += sbytes;
  pl.off_acc = off; off += align_up(static_cast<size_t>(n) * pl.wpad * sizeof(float));
  pl.off_part = off; off += align_up(static_cast<size_t>(J + 1) * 2 * nb * sizeof(double));
  pl.off_mom = off; off += align_up(static_cast<size_t>(J + 1) * 2 * sizeof(double));
  pl.total = off;
  return pl;
}

// Workspace large enough for every variant and for moments up to degree m_max.
size_t filter_workspace(int64_t n, int w, csc_dtype iter_dt, int m_max) {
  size_t best = 0;
  for (int v = 0; v < num_variants(); ++v)
    best = std::max(best, make_plan(n, w, iter_dt, v, m_max).total);
  return best;
}

static double step_bytes(const Graph* g, int64_t n, int w, csc_dtype iter_dt, int flags,
                         csc_dtype y_dt) {
  const double sz = static_cast<double>(dtype_size(iter_dt));
  const double ss = iter_split(iter_dt) ? 4.0 : sz;  // state element (own-row streams)
  double b = static_cast<double>(g->nnz) * (4.0 + dtype_size(g->val_dt)) + 4.0 * (n + 1);
  if (g->diag) b += 4.0 * n;                      // degrees (combinatorial)
  const double nw = static_cast<double>(n) * w;
  b += nw * sz;                                   // gather Z_j (each row counted once)
  if ((flags & F_OWN) && iter_split(iter_dt)) b += nw * ss;  // own Z_j from the state
  if (!(flags & F_FIRST)) b += nw * ss;           // Z_{j-1}
  if (flags & F_STORE) b += nw * (iter_split(iter_dt) ? ss + sz : sz);  // Z_{j+1}
  if (flags & F_ACC) b += nw * 4.0 + ((flags & F_LAST) ? nw * dtype_size(y_dt) : nw * 4.0);
  return b;
}

csc_status run_filter(const Graph* g, double lmax, int m, const double* a, const void* X,
                      csc_dtype x_dt, int64_t ldx, void* Y, csc_dtype y_dt, int64_t ldy, int w,
                      csc_dtype iter_dt, double* moments, int moments_only, void* work,
                      size_t work_bytes, hipStream_t s, int variant_override) {
  const int64_t n = g->n;
  if (m < 0) return fail(CSC_E_ARG, "m must be >= 0");
  if (w < 1) return fail(CSC_E_ARG, "w must be >= 1");
  if (!(lmax > 0.0)) return fail(CSC_E_ARG, "lmax must be > 0");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "iterates must be F32, BF16, F16, BF16S or F16S");
  if (moments && m < 1) return fail(CSC_E_ARG, "moments need m >= 1");
  if (!moments_only && (ldy < w || !Y)) return fail(CSC_E_ARG, "bad Y / ldy");
  if (ldx < w || !X) return fail(CSC_E_ARG, "bad X / ldx");
  if (!moments_only) {
    const char* xb = static_cast<const char*>(X);
    const char* yb = static_cast<const char*>(Y);
    const size_t xspan = (static_cast<size_t>(n - 1) * ldx + w) * dtype_size(x_dt);
    const size_t yspan = (static_cast<size_t>(n - 1) * ldy + w) * dtype_size(y_dt);
    if (n > 0 && xb < yb + yspan && yb < xb + xspan)
      return fail(CSC_E_ARG, "X and Y overlap");
  }
  if (n == 0) return CSC_OK;
  const int variant = variant_override >= 0 ? variant_override : default_variant(g, w, iter_dt);
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, moments ? m : 0);
  if (!work || work_bytes < pl.total)
    return fail(CSC_E_ARG, "workspace too small: need " + std::to_string(pl.total) + " bytes");
  char* base = static_cast<char*>(work);
  void* zb[2] = {base + pl.off_z0, base + pl.off_z1};
  float* sb[2] = {reinterpret_cast<float*>(base + pl.off_s0), reinterpret_cast<float*>(base + pl.off_s1)};
  float* acc = reinterpret_cast<float*>(base + pl.off_acc);
  double* part = reinterpret_cast<double*>(base + pl.off_part);
  double* msum = reinterpret_cast<double*>(base + pl.off_mom);
  const int wt = pl.shape.wt();
  const bool do_acc = !moments_only;

  launch_init(iter_dt, X, x_dt, ldx, n, w, pl.wpad, wt, zb[0], do_acc ? acc : nullptr,
              static_cast<float>(a ? a[0] : 0.0), sb[0], s);
  CSC_HIP(hipGetLastError());
  if (m == 0) {
    if (do_acc) {
      const int64_t total = n * w;
      hipLaunchKernelGGL(k_acc_out, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                         0, s, acc, n, w, pl.wpad, Y, int(y_dt), ldy);
      CSC_HIP(hipGetLastError());
    }
    return CSC_OK;
  }

  const StepFn fn = step_fn(iter_dt, pl.shape.lpr, g->val_dt);
  const int64_t nb = pl.row_blocks * pl.ntiles;
  const int J = moments ? m / 2 : -1;
  const int nsteps = moments_only ? J + 1 : m;
  const OpScale op = op_scale(g, lmax);
  double bytes = 0.0;
  timing_begin(s);
  for (int j = 0; j < nsteps; ++j) {
    StepParams p{};
    p.rowptr = g->rowptr;
    p.colidx = g->colidx;
    p.vals = g->vals;
    p.zcur = zb[j & 1];
    p.zprev = zb[(j + 1) & 1];
    p.zout = zb[(j + 1) & 1];
    p.scur = sb[j & 1];
    p.sprev = sb[(j + 1) & 1];
    p.sout = sb[(j + 1) & 1];
    p.acc = acc;
    p.ld_acc = pl.wpad;
    p.w = w;
    p.n = n;
    p.row_blocks = pl.row_blocks;
    set_op(p, op);
    p.coef = static_cast<float>(do_acc ? a[j + 1] : 0.0);
    const bool last = j == nsteps - 1;
    const bool mom = moments && j <= J;
    int flags = 0;
    if (j == 0) flags |= F_FIRST;
    if (do_acc) flags |= F_ACC;
    if (do_acc && last) {
      flags |= F_LAST;
      p.yout = Y;
      p.ldy = ldy;
      p.y_dt = int(y_dt);
    }
    if (mom) {
      flags |= F_MOM;
      p.mom_part = part + static_cast<int64_t>(j) * 2 * nb;
    }
    if (!last) flags |= F_STORE;
    if (mom || op.own()) flags |= F_OWN;
    p.flags = flags;
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, p);
    bytes += step_bytes(g, n, w, iter_dt, flags, y_dt);
  }
  timing_end(s, nsteps, bytes);
  CSC_HIP(hipGetLastError());
  if (moments) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(2 * (J + 1)), dim3(kThreads), 0, s, part, nb, msum);
    hipLaunchKernelGGL(k_moments, dim3(1), dim3(64), 0, s, msum, J, m, moments);
    CSC_HIP(hipGetLastError());
  }
  return CSC_OK;
}

}  // namespace csc

// =====================================================================================
// Adjoint of the filter (reverse mode).  With Zb_j = dl/dZ_j and Zb_{m+1} = Zb_{m+2} = 0:
//     Zb_j = a_j G + f_j (alpha Zb_{j+1} - beta A^T Zb_{j+1}) - Zb_{j+2},  f_j = 2 (j >= 1), 1 (j = 0)
//     dl/dA_e += -beta f_j <Zb_{j+1}[r], Z_j[c]>   for every stored entry e = (r, c)
//     dl/da_j  = <G, Z_j>,   dl/dX = Zb_0.
// The forward iterates are recomputed segment by segment from checkpoint pairs
// (Z_s, Z_{s+1}) taken every `ckpt` steps.  The fused adjoint kernel gathers Zb_{j+1} and
// Z_j over the same CSR entries (transposed product and sampled dense-dense product) and
// loops over the column tiles inside the block, so each entry's gradient is accumulated
// by one lane in a fixed order.
namespace csc {

namespace {

struct AdjParams {
  const int32_t* rowptr;
  const int32_t* colidx;
  const void* valsT;   // A^T values on A's pattern
  const float* zb1;    // Zb_{j+1}, tiled
  const float* zb2;    // Zb_{j+2}, tiled, or null (zero)
  float* zbout;        // Zb_j, tiled (may alias zb2)
  const float* zj;     // Z_j, tiled
  const float* G;      // row-major, ldg
  int64_t ldg;
  float* dA;           // nnz
  int64_t n;
  int w, ntiles;
  float alpha, beta, aj, fac, sdd;
};

template <typename TV, int LPR>
__global__ __launch_bounds__(kThreads) void k_adj(AdjParams p) {
  constexpr int VEC = 4;
  constexpr int WT = LPR * VEC;
  constexpr int RPB = kThreads / LPR;
  __shared__ int32_t s_col[kStageCap];
  __shared__ float s_val[kStageCap];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RPB;
  const int64_t r1 = min(r0 + RPB, p.n);
  const int32_t e0 = p.rowptr[r0];
  const int32_t cnt = p.rowptr[r1] - e0;
  const bool staged = cnt <= kStageCap;
  const TV* vals = static_cast<const TV*>(p.valsT);
  if (staged)
    for (int32_t i = threadIdx.x; i < cnt; i += kThreads) {
      s_col[i] = p.colidx[e0 + i];
      s_val[i] = val_f<TV>(vals[e0 + i]);
    }
  __syncthreads();
  const int64_t row = r0 + threadIdx.x / LPR;
  const int lane = threadIdx.x % LPR;
  if (row >= p.n) return;
  const int32_t rs = p.rowptr[row], re = p.rowptr[row + 1];
  for (int tile = 0; tile < p.ntiles; ++tile) {
    const int64_t toff = static_cast<int64_t>(tile) * p.n * WT + lane * VEC;
    const float* zb1 = p.zb1 + toff;
    const float* zj = p.zj + toff;
    float ob[VEC], acc[VEC];
    Pack<float>::unpack(ld16(zb1 + row * WT), ob);
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc[i] = 0.f;
    for (int32_t e = rs; e < re; ++e) {
      const int32_t c = staged ? s_col[e - e0] : p.colidx[e];
      const float v = staged ? s_val[e - e0] : val_f<TV>(vals[e]);
      float gb[VEC], gz[VEC];
      Pack<float>::unpack(ld16(zb1 + static_cast<int64_t>(c) * WT), gb);
      Pack<float>::unpack(ld16(zj + static_cast<int64_t>(c) * WT), gz);
      float sd = 0.f;
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        acc[i] = fmaf(v, gb[i], acc[i]);
        sd = fmaf(ob[i], gz[i], sd);
      }
#pragma unroll
      for (int off = LPR / 2; off > 0; off >>= 1) sd += __shfl_xor(sd, off, LPR);
      if (p.dA && lane == 0) p.dA[e] += p.sdd * sd;
    }
    const int64_t col0 = static_cast<int64_t>(tile) * WT + lane * VEC;
    float out[VEC];
    float z2[VEC];
    if (p.zb2) Pack<float>::unpack(ld16(p.zb2 + toff + row * WT), z2);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      const float g = (col0 + i < p.w) ? p.G[row * p.ldg + col0 + i] : 0.f;
      out[i] = fmaf(p.aj, g, p.fac * fmaf(p.alpha, ob[i], -p.beta * acc[i]));
      if (p.zb2) out[i] -= z2[i];
    }
    st16(p.zbout + toff + row * WT, Pack<float>::pack(out));
  }
}

// Zb = s * G in the tiled layout (zero in padded columns).
__global__ void k_scale_tiled(const float* G, int64_t ldg, int64_t n, int w, int wpad, int wt,
                              float s, float* out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * wpad) return;
  const int64_t row = idx / wpad;
  const int col = static_cast<int>(idx - row * wpad);
  const int tile = col / wt, c = col - tile * wt;
  out[static_cast<int64_t>(tile) * n * wt + row * wt + c] = col < w ? s * G[row * ldg + col] : 0.f;
}

// Row-major out (ld) from the tiled layout.
__global__ void k_tiled_out(const float* Z, int64_t n, int w, int wt, float* out, int64_t ld) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * w) return;
  const int64_t row = idx / w;
  const int col = static_cast<int>(idx - row * w);
  const int tile = col / wt, c = col - tile * wt;
  out[row * ld + col] = Z[static_cast<int64_t>(tile) * n * wt + row * wt + c];
}

// Block partials of <G, Z> with Z tiled (FP64, fixed order).
__global__ void k_gdot_part(const float* Z, const float* G, int64_t ldg, int64_t n, int w, int wt,
                            double* part) {
  const int64_t total = n * w;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  double s = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
    const int64_t row = i / w;
    const int col = static_cast<int>(i - row * w);
    const int tile = col / wt, c = col - tile * wt;
    s += static_cast<double>(G[row * ldg + col]) *
         static_cast<double>(Z[static_cast<int64_t>(tile) * n * wt + row * wt + c]);
  }
  double dummy = 0.0;
  block_reduce2(s, dummy);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename TV>
__global__ void k_transpose_vals(const TV* vals, const int32_t* mirror, int64_t nnz, TV* out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) out[e] = vals[mirror[e]];
}

__global__ void k_zero(float* p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

using AdjFn = void (*)(AdjParams);
AdjFn pick_adj(int lpr, csc_dtype val_dt) {
  const bool vb = val_dt == CSC_BF16;
  switch (lpr) {
    case 4: return vb ? k_adj<uint16_t, 4> : k_adj<float, 4>;
    case 8: return vb ? k_adj<uint16_t, 8> : k_adj<float, 8>;
    case 16: return vb ? k_adj<uint16_t, 16> : k_adj<float, 16>;
    default: return vb ? k_adj<uint16_t, 32> : k_adj<float, 32>;
  }
}

constexpr int64_t kGdotBlocks = 1024;

struct BwdLayout {
  FilterPlan pl;
  int ckpt, nseg;
  size_t zbytes;
  size_t off_ckpt, off_seg, off_pp, off_zb, off_vt, off_part, total;
};

BwdLayout bwd_layout(int64_t n, int w, int m, int ckpt, int variant, size_t nnz_cap) {
  BwdLayout L{};
  L.pl = make_plan(n, w, CSC_F32, variant, 0);
  if (ckpt <= 0) ckpt = std::max(2, static_cast<int>(std::ceil(std::sqrt(static_cast<double>(std::max(m, 1))))));
  L.ckpt = std::max(2, ckpt);
  L.nseg = std::max(1, (m + L.ckpt - 1) / L.ckpt);
  L.zbytes = align_up(static_cast<size_t>(n) * L.pl.wpad * sizeof(float));
  size_t off = 0;
  L.off_ckpt = off; off += 2 * L.nseg * L.zbytes;
  L.off_seg = off; off += (L.ckpt - 2 > 0 ? L.ckpt - 2 : 0) * L.zbytes;
  L.off_pp = off; off += 2 * L.zbytes;   // forward ping-pong
  L.off_zb = off; off += 2 * L.zbytes;   // adjoint pair
  L.off_vt = off; off += align_up(nnz_cap * 4);
  L.off_part = off; off += align_up(static_cast<size_t>(m + 1) * kGdotBlocks * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

size_t backward_workspace(int64_t n, int w, int m, int ckpt) {
  // the transposed values need the graph's capacity; callers size it with nnz = 64 n at most
  size_t best = 0;
  for (int v = 0; v < num_variants(); ++v)
    best = std::max(best, bwd_layout(n, w, m, ckpt, v, static_cast<size_t>(n) * 64).total);
  return best;
}

csc_status run_backward(const Graph* g, double lmax, int m, const double* a, const float* X,
                        int64_t ldx, const float* G, int64_t ldg, int w, float* dX, int64_t lddx,
                        double* da, float* dA, int ckpt, void* work, size_t work_bytes,
                        hipStream_t s) {
  const int64_t n = g->n;
  if (m < 0 || m > 4096) return fail(CSC_E_ARG, "m must be in [0, 4096]");
  if (w < 1 || ldx < w || ldg < w || (dX && lddx < w)) return fail(CSC_E_ARG, "bad sizes");
  if (!(lmax > 0.0)) return fail(CSC_E_ARG, "lmax must be > 0");
  if (g->nnz > n * 64) return fail(CSC_E_ARG, "backward supports nnz <= 64 n");
  const int variant = default_variant(g, w, CSC_F32);
  const BwdLayout L = bwd_layout(n, w, m, ckpt, variant, static_cast<size_t>(std::max<int64_t>(g->nnz, 1)));
  if (!work || work_bytes < L.total)
    return fail(CSC_E_ARG, "backward workspace too small: need " + std::to_string(L.total));
  const FilterPlan& pl = L.pl;
  const int wt = pl.shape.wt();
  char* base = static_cast<char*>(work);
  auto ck = [&](int q, int which) {
    return reinterpret_cast<float*>(base + L.off_ckpt + (2 * q + which) * L.zbytes);
  };
  auto seg = [&](int i) { return reinterpret_cast<float*>(base + L.off_seg + (i - 2) * L.zbytes); };
  float* pp[2] = {reinterpret_cast<float*>(base + L.off_pp),
                  reinterpret_cast<float*>(base + L.off_pp + L.zbytes)};
  float* zbb[2] = {reinterpret_cast<float*>(base + L.off_zb),
                   reinterpret_cast<float*>(base + L.off_zb + L.zbytes)};
  void* valsT = base + L.off_vt;
  double* part = reinterpret_cast<double*>(base + L.off_part);
  const size_t tiled_bytes = static_cast<size_t>(n) * pl.wpad * sizeof(float);
  const unsigned eblocks = static_cast<unsigned>((n * pl.wpad + 255) / 256);
  if (g->lap != CSC_LAP_NORMALIZED) return fail(CSC_E_ARG, "the adjoint is defined for the normalized Laplacian");
  const OpScale op = op_scale(g, lmax);
  const float alpha = op.alpha;
  const float beta = op.beta;
  const int64_t nb = pl.row_blocks * pl.ntiles;
  const StepFn fstep = pick_step<float>(pl.shape.lpr, g->val_dt);
  const int gblocks = static_cast<int>(std::min<int64_t>(kGdotBlocks, std::max<int64_t>(1, (n * w + kThreads - 1) / kThreads)));

  if (n == 0) return CSC_OK;
  // transposed values on A's pattern
  if (g->nnz > 0) {
    const unsigned vb = static_cast<unsigned>((g->nnz + 255) / 256);
    if (g->val_dt == CSC_F32)
      hipLaunchKernelGGL(k_transpose_vals<float>, dim3(vb), dim3(256), 0, s,
                         static_cast<const float*>(g->vals), g->mirror, g->nnz, static_cast<float*>(valsT));
    else
      hipLaunchKernelGGL(k_transpose_vals<uint16_t>, dim3(vb), dim3(256), 0, s,
                         static_cast<const uint16_t*>(g->vals), g->mirror, g->nnz,
                         static_cast<uint16_t*>(valsT));
  }
  if (dA && g->nnz > 0)
    hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>((g->nnz + 255) / 256)), dim3(256), 0, s, dA, g->nnz);

  auto step = [&](const float* zcur, const float* zprev, float* zout, bool first) {
    StepParams p{};
    p.rowptr = g->rowptr;
    p.colidx = g->colidx;
    p.vals = g->vals;
    p.zcur = zcur;
    p.zprev = zprev;
    p.zout = zout;
    p.n = n;
    p.w = w;
    p.row_blocks = pl.row_blocks;
    set_op(p, op);
    p.flags = F_STORE | (first ? F_FIRST : 0) | (op.own() ? F_OWN : 0);
    hipLaunchKernelGGL(fstep, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, p);
  };
  auto gdot = [&](const float* Z, int j) {
    hipLaunchKernelGGL(k_gdot_part, dim3(gblocks), dim3(kThreads), 0, s, Z, G, ldg, n, w, wt,
                       part + static_cast<int64_t>(j) * gblocks);
  };

  // ---- forward with checkpoints: Z_0 .. Z_m in the ping-pong pair (Z_{j+1} overwrites
  // Z_{j-1} in place), copies of Z_i into the checkpoint slots when i = q ckpt or q ckpt + 1,
  // and da_j = <G, Z_j>
  auto keep = [&](int i, const float* z) -> csc_status {
    const int q = i / L.ckpt, r = i % L.ckpt;
    if (q < L.nseg && r <= 1)
      CSC_HIP(hipMemcpyAsync(ck(q, r), z, tiled_bytes, hipMemcpyDeviceToDevice, s));
    return CSC_OK;
  };
  hipLaunchKernelGGL(k_init<float>, dim3(eblocks), dim3(256), 0, s, static_cast<const void*>(X),
                     int(CSC_F32), ldx, n, w, pl.wpad, wt, pp[0], static_cast<float*>(nullptr), 0.f,
                     static_cast<float*>(nullptr), static_cast<const double*>(nullptr));
  gdot(pp[0], 0);
  CSC_TRY(keep(0, pp[0]));
  for (int j = 0; j < m; ++j) {
    step(pp[j & 1], pp[(j + 1) & 1], pp[(j + 1) & 1], j == 0);
    gdot(pp[(j + 1) & 1], j + 1);
    CSC_TRY(keep(j + 1, pp[(j + 1) & 1]));
  }
  if (da) hipLaunchKernelGGL(k_reduce_rows, dim3(m + 1), dim3(kThreads), 0, s, part, int64_t(gblocks), da);

  // ---- reverse sweep
  hipLaunchKernelGGL(k_scale_tiled, dim3(eblocks), dim3(256), 0, s, G, ldg, n, w, pl.wpad, wt,
                     static_cast<float>(a[m]), zbb[0]);
  const float* zb1 = zbb[0];  // Zb_{j+1}
  const float* zb2 = nullptr; // Zb_{j+2}
  const AdjFn adj = pick_adj(pl.shape.lpr, g->val_dt);
  for (int q = (m >= 1 ? (m - 1) / L.ckpt : -1); q >= 0; --q) {
    const int s0 = q * L.ckpt;
    const int s1 = std::min(s0 + L.ckpt - 1, m - 1);  // segment iterates Z_s0 .. Z_s1
    auto Zp = [&](int j) -> const float* {
      const int i = j - s0;
      if (i == 0) return ck(q, 0);
      if (i == 1) return ck(q, 1);
      return seg(i);
    };
    for (int j = s0 + 2; j <= s1; ++j) step(Zp(j - 1), Zp(j - 2), seg(j - s0), false);
    for (int j = s1; j >= s0; --j) {
      AdjParams p{};
      p.rowptr = g->rowptr;
      p.colidx = g->colidx;
      p.valsT = valsT;
      p.zb1 = zb1;
      p.zb2 = zb2;
      float* out = zb2 ? const_cast<float*>(zb2) : (zb1 == zbb[0] ? zbb[1] : zbb[0]);
      p.zbout = out;
      p.zj = Zp(j);
      p.G = G;
      p.ldg = ldg;
      p.dA = dA;
      p.n = n;
      p.w = w;
      p.ntiles = pl.ntiles;
      p.alpha = alpha;
      p.beta = beta;
      p.aj = static_cast<float>(a[j]);
      p.fac = j >= 1 ? 2.f : 1.f;
      p.sdd = -beta * p.fac;
      hipLaunchKernelGGL(adj, dim3(static_cast<unsigned>(pl.row_blocks)), dim3(kThreads), 0, s, p);
      zb2 = zb1;
      zb1 = out;
    }
  }
  // zb1 now holds Zb_0 (for m == 0 it holds a_0 G)
  if (dX)
    hipLaunchKernelGGL(k_tiled_out, dim3(static_cast<unsigned>((n * w + 255) / 256)), dim3(256), 0, s,
                       zb1, n, w, wt, dX, lddx);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace csc

// =====================================================================================
// Stored basis.  The iterates Z_j = T_j(L~) X, j = 0..m, of one block are all kept (tiled
// layout, one slot per j), so the filter at any cut-off is the linear combination
// Y = sum_j a_j Z_j and the Chebyshev moments follow from dot products of stored iterates;
// a change of cut-off then costs one streaming pass instead of a new recurrence.
namespace csc {

namespace {

constexpr int kMaxCombine = 256;  // FP64 coefficients in the 4 KiB kernel arguments

struct CombineParams {
  const void* basis;   // (m + 1) slots of n x wpad (tiled)
  int64_t slot;        // elements per slot
  int64_t n;
  int w, wt, wpad, m;
  void* Y;
  int y_dt;
  int64_t ldy;
  const void* P;       // optional: <P, Y> partials
  int p_dt;
  int64_t ldp;
  int vec;             // Y (and P) in whole 16-byte pieces per lane: vector stores and loads
  double* part;        // per block
  double coef[kMaxCombine];
};

__device__ inline float load_any(const void* p, int dt, int64_t i) {
  if (dt == CSC_F32) return static_cast<const float*>(p)[i];
  if (dt == CSC_BF16) return bf16_to_f32(static_cast<const uint16_t*>(p)[i]);
  return static_cast<float>(static_cast<const double*>(p)[i]);
}

// One thread per (row, VEC columns of a tile): Y = sum_j a_j Z_j with FP64 coefficients,
// accumulated in FP64 in the order j = 0..m and rounded once.  The filtered block can be a
// small fraction of the input's norm (about 0.2% at the C3 cut-off), so FP32 coefficients
// and an FP32 sum would cost more accuracy than the iterates themselves carry.
template <typename TZ>
__global__ __launch_bounds__(kThreads) void k_combine(CombineParams p) {
  constexpr int VEC = Pack<TZ>::VEC;
  const int lanes_per_row = p.wpad / VEC;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  double dot = 0.0;
  if (t < p.n * lanes_per_row) {
    const int64_t row = t / lanes_per_row;
    const int q = static_cast<int>(t - row * lanes_per_row);
    const int col0 = q * VEC;
    const int tile = col0 / p.wt, c = col0 - tile * p.wt;
    const TZ* z = static_cast<const TZ*>(p.basis) + static_cast<int64_t>(tile) * p.n * p.wt +
                  row * p.wt + c;
    // the lane's probe values, read ahead of the slot loop on the vector path (F32 or BF16
    // pieces, 4 or 8 values each)
    constexpr int PW = VEC / 4;
    uint4 praw[PW];
    const bool vp = p.vec && p.P && col0 < p.w;
    if (vp) {
      const char* pb = static_cast<const char*>(p.P) +
                       (row * p.ldp + col0) * static_cast<int64_t>(p.p_dt == CSC_BF16 ? 2 : 4);
#pragma unroll
      for (int w = 0; w < PW; ++w)
        praw[w] = (p.p_dt == CSC_BF16 && w > 0) ? praw[0] : ld16(pb + 16 * w);
    }
    double y[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) y[i] = 0.0;
    // eight slots' loads in flight, then their terms in slot order
    constexpr int JU = 8;
    int j = 0;
    for (; j + JU <= p.m + 1; j += JU) {
      uint4 g[JU];
#pragma unroll
      for (int u = 0; u < JU; ++u) g[u] = ld16(z + static_cast<int64_t>(j + u) * p.slot);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < JU; ++u) {
        float f[VEC];
        Pack<TZ>::unpack(g[u], f);
        const double a = p.coef[j + u];
#pragma unroll
        for (int i = 0; i < VEC; ++i) y[i] = fma(a, static_cast<double>(f[i]), y[i]);
      }
    }
    for (; j <= p.m; ++j) {
      float f[VEC];
      Pack<TZ>::unpack(ld16(z + static_cast<int64_t>(j) * p.slot), f);
      const double a = p.coef[j];
#pragma unroll
      for (int i = 0; i < VEC; ++i) y[i] = fma(a, static_cast<double>(f[i]), y[i]);
    }
    if (p.vec) {
      if (col0 < p.w) {
        float y32[VEC], yv[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) y32[i] = static_cast<float>(y[i]);
        char* yb = static_cast<char*>(p.Y) + (row * p.ldy + col0) *
                                               static_cast<int64_t>(p.y_dt == CSC_BF16 ? 2 : 4);
        if (p.y_dt == CSC_BF16) {
#pragma unroll
          for (int i0 = 0; i0 < VEC; i0 += 8) {
            uint32_t wd[4];
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
              const uint16_t lo = f32_to_bf16(y32[i0 + 2 * k2]), hi = f32_to_bf16(y32[i0 + 2 * k2 + 1]);
              yv[i0 + 2 * k2] = bf16_to_f32(lo);
              yv[i0 + 2 * k2 + 1] = bf16_to_f32(hi);
              wd[k2] = static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 16);
            }
            st16(yb + 2 * i0, make_uint4(wd[0], wd[1], wd[2], wd[3]));
          }
        } else {
#pragma unroll
          for (int i0 = 0; i0 < VEC; i0 += 4) {
            st16(yb + 4 * i0, make_uint4(__float_as_uint(y32[i0]), __float_as_uint(y32[i0 + 1]),
                                         __float_as_uint(y32[i0 + 2]), __float_as_uint(y32[i0 + 3])));
#pragma unroll
            for (int i = 0; i < 4; ++i) yv[i0 + i] = y32[i0 + i];
          }
        }
        if (vp) {
          float pv[VEC];
          if (p.p_dt == CSC_BF16) {
            // eight BF16 values per piece (VEC = 8 here: BF16 probes go with BF16 copies)
            const uint32_t wd[4] = {praw[0].x, praw[0].y, praw[0].z, praw[0].w};
#pragma unroll
            for (int i = 0; i < VEC; ++i)
              pv[i] = i < 8 ? __uint_as_float(i & 1 ? wd[(i >> 1) & 3] & 0xffff0000u : wd[(i >> 1) & 3] << 16)
                            : 0.f;
          } else {
#pragma unroll
            for (int w = 0; w < PW; ++w) {
              pv[4 * w] = __uint_as_float(praw[w].x); pv[4 * w + 1] = __uint_as_float(praw[w].y);
              pv[4 * w + 2] = __uint_as_float(praw[w].z); pv[4 * w + 3] = __uint_as_float(praw[w].w);
            }
          }
#pragma unroll
          for (int i = 0; i < VEC; ++i) dot += static_cast<double>(pv[i]) * static_cast<double>(yv[i]);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        const int col = col0 + i;
        if (col < p.w) {
          const float y32 = static_cast<float>(y[i]);
          float yv = y32;
          if (p.y_dt == CSC_BF16) yv = bf16_to_f32(f32_to_bf16(yv));
          store_out(p.Y, p.y_dt, row * p.ldy + col, y32);
          if (p.P) dot += static_cast<double>(load_any(p.P, p.p_dt, row * p.ldp + col)) * static_cast<double>(yv);
        }
      }
    }
  }
  if (p.part) {
    double dummy = 0.0;
    block_reduce2(dot, dummy);
    if (threadIdx.x == 0) p.part[blockIdx.x] = dot;
  }
}

// Direct moments from the kept basis: part[j * gridDim.x + b] = block b's share of
// <Z_0, Z_j> (FP64, fixed order).  Z_0 is the probe block itself, so the rounding of the
// stored Z_j enters only through <P, e_j>, which has zero mean; the doubled form
// 2 <Z_j, Z_j> - mu_0 would instead carry the positive bias 2 ||e_j||^2.  Each thread keeps
// kDirV 16-byte vectors of Z_0 in registers while it walks the m + 1 slots, so every slot is
// read once (padded columns are zero in both).
constexpr int kDirV = 4;

template <typename TZ>
__global__ __launch_bounds__(kThreads) void k_dir_moments(const TZ* basis, int64_t slot,
                                                          int64_t nvec, int m, double* part) {
  constexpr int VEC = Pack<TZ>::VEC;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kDirV + threadIdx.x;
  float z0[kDirV][VEC];
#pragma unroll
  for (int q = 0; q < kDirV; ++q) {
    const int64_t v = base + q * kThreads;
    if (v < nvec) Pack<TZ>::unpack(ld16(basis + v * VEC), z0[q]);
    else
#pragma unroll
      for (int i = 0; i < VEC; ++i) z0[q][i] = 0.f;
  }
  for (int j = 0; j <= m; ++j) {
    const TZ* zj = basis + static_cast<int64_t>(j) * slot;
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < kDirV; ++q) {
      const int64_t v = base + q * kThreads;
      if (v < nvec) {
        float f[VEC];
        Pack<TZ>::unpack(ld16(zj + v * VEC), f);
        float sp = 0.f;
#pragma unroll
        for (int i = 0; i < VEC; ++i) sp = fmaf(z0[q][i], f[i], sp);
        d += static_cast<double>(sp);
      }
    }
    double dummy = 0.0;
    block_reduce2(d, dummy);
    if (threadIdx.x == 0) part[static_cast<int64_t>(j) * gridDim.x + blockIdx.x] = d;
  }
}

}  // namespace

// m + 1 slots of the stored iterates, then (BF16S) the two FP32 state buffers.
size_t basis_bytes(int64_t n, int w, int m, csc_dtype iter_dt, int variant) {
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  return static_cast<size_t>(m + 1) * align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt)) +
         2 * align_up(static_cast<size_t>(n) * pl.wpad * state_size(iter_dt));
}

static int64_t dir_blocks(int64_t n, int w, csc_dtype iter_dt, int variant, int64_t* nvec) {
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  const int VEC = iter_dt == CSC_F32 ? 4 : 8;
  *nvec = n * (pl.wpad / VEC);
  return std::max<int64_t>(1, (*nvec + kThreads * kDirV - 1) / (kThreads * kDirV));
}

// Scratch of the recombination dot and of the direct moments.
size_t basis_aux_bytes(int64_t n, int w, int m, csc_dtype iter_dt, int variant) {
  int64_t nvec = 0;
  const int64_t nb = dir_blocks(n, w, iter_dt, variant, &nvec);
  const size_t moments = align_up(static_cast<size_t>(m + 1) * nb * sizeof(double));
  const size_t combine = align_up(static_cast<size_t>((nvec + kThreads - 1) / kThreads + 1) * sizeof(double));
  return std::max(moments, combine);
}

csc_status run_basis(const Graph* g, double lmax, int m, const void* X, csc_dtype x_dt, int64_t ldx,
                     int w, csc_dtype iter_dt, int variant, void* basis, size_t bytes, hipStream_t s) {
  const int64_t n = g->n;
  if (m < 1 || w < 1 || ldx < w || !X) return fail(CSC_E_ARG, "bad basis arguments");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "iterates must be F32, BF16, F16, BF16S or F16S");
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  const size_t slot_bytes = align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt));
  const size_t state_bytes = align_up(static_cast<size_t>(n) * pl.wpad * state_size(iter_dt));
  if (!basis || bytes < basis_bytes(n, w, m, iter_dt, variant)) return fail(CSC_E_ARG, "basis buffer too small");
  char* b = static_cast<char*>(basis);
  float* st[2] = {reinterpret_cast<float*>(b + static_cast<size_t>(m + 1) * slot_bytes),
                  reinterpret_cast<float*>(b + static_cast<size_t>(m + 1) * slot_bytes + state_bytes)};
  const int wt = pl.shape.wt();
  launch_init(iter_dt, X, x_dt, ldx, n, w, pl.wpad, wt, b, nullptr, 0.f, st[0], s);
  const StepFn fn = step_fn(iter_dt, pl.shape.lpr, g->val_dt);
  const int64_t nb = pl.row_blocks * pl.ntiles;
  const OpScale op = op_scale(g, lmax);
  double bytes_alg = 0.0;
  timing_begin(s);
  for (int j = 0; j < m; ++j) {
    StepParams p{};
    p.rowptr = g->rowptr;
    p.colidx = g->colidx;
    p.vals = g->vals;
    p.zcur = b + static_cast<size_t>(j) * slot_bytes;
    p.zprev = j > 0 ? b + static_cast<size_t>(j - 1) * slot_bytes : nullptr;
    p.zout = b + static_cast<size_t>(j + 1) * slot_bytes;
    p.scur = st[j & 1];
    p.sprev = st[(j + 1) & 1];
    p.sout = st[(j + 1) & 1];
    p.w = w;
    p.n = n;
    p.row_blocks = pl.row_blocks;
    set_op(p, op);
    p.flags = F_STORE | (j == 0 ? F_FIRST : 0) | (op.own() ? F_OWN : 0);
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s, p);
    bytes_alg += step_bytes(g, n, w, iter_dt, p.flags, CSC_F32);
  }
  timing_end(s, m, bytes_alg);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// Y = sum_j a_j Z_j from the stored basis; when P is given, *dot (device) = <P, Y> with Y as
// stored (rounded to y_dt).
csc_status run_combine(const void* basis, int64_t n, int w, int m, csc_dtype iter_dt, int variant,
                       const double* a, void* Y, csc_dtype y_dt, int64_t ldy, const void* P,
                       csc_dtype p_dt, int64_t ldp, double* dot, void* aux, size_t aux_bytes,
                       hipStream_t s) {
  if (m + 1 > kMaxCombine) return fail(CSC_E_ARG, "combine supports m < 256");
  if (!Y || ldy < w) return fail(CSC_E_ARG, "bad Y");
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  const int VEC = iter_dt == CSC_F32 ? 4 : 8;  // the 16-bit modes keep 16-bit copies
  const int64_t threads = n * (pl.wpad / VEC);
  const unsigned blocks = static_cast<unsigned>((threads + kThreads - 1) / kThreads);
  if (dot && aux_bytes < align_up((blocks + 1) * sizeof(double))) return fail(CSC_E_ARG, "aux too small");
  CombineParams p{};
  p.basis = basis;
  p.slot = static_cast<int64_t>(align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt)) / dtype_size(iter_dt));
  p.n = n;
  p.w = w;
  p.wt = pl.shape.wt();
  p.wpad = pl.wpad;
  p.m = m;
  p.Y = Y;
  p.y_dt = int(y_dt);
  p.ldy = ldy;
  p.P = dot ? P : nullptr;
  p.p_dt = int(p_dt);
  p.ldp = ldp;
  p.part = dot ? static_cast<double*>(aux) : nullptr;
  // vector epilogue: whole pieces per lane (w a multiple of VEC), 16-byte aligned rows, and
  // element types whose pieces match the lane's VEC values (BF16 only with eight per lane)
  auto rows16 = [](const void* b, int64_t ld, csc_dtype dt) {
    return reinterpret_cast<uintptr_t>(b) % 16 == 0 && (ld * static_cast<int64_t>(dtype_size(dt))) % 16 == 0;
  };
  auto type_ok = [&](csc_dtype dt) { return dt == CSC_F32 || (dt == CSC_BF16 && VEC == 8); };
  p.vec = (w % VEC == 0 && type_ok(y_dt) && rows16(Y, ldy, y_dt) &&
           (!p.P || (type_ok(p_dt) && rows16(P, ldp, p_dt)))) ? 1 : 0;
  for (int j = 0; j <= m; ++j) p.coef[j] = a[j];
  if (iter_dt == CSC_F32)
    hipLaunchKernelGGL(k_combine<float>, dim3(blocks), dim3(kThreads), 0, s, p);
  else if (iter_half(iter_dt))
    hipLaunchKernelGGL(k_combine<_Float16>, dim3(blocks), dim3(kThreads), 0, s, p);
  else
    hipLaunchKernelGGL(k_combine<uint16_t>, dim3(blocks), dim3(kThreads), 0, s, p);
  if (dot) hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kThreads), 0, s, static_cast<double*>(aux),
                              static_cast<int64_t>(blocks), dot);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// mu_0..mu_m (device) of the stored basis in the direct form mu_j = <Z_0, Z_j>.
csc_status run_basis_moments(const void* basis, int64_t n, int w, int m, csc_dtype iter_dt,
                             int variant, double* moments, void* aux, size_t aux_bytes,
                             hipStream_t s) {
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  int64_t nvec = 0;
  const int64_t nb = dir_blocks(n, w, iter_dt, variant, &nvec);
  if (aux_bytes < static_cast<size_t>(m + 1) * nb * sizeof(double)) return fail(CSC_E_ARG, "aux too small");
  double* part = static_cast<double*>(aux);
  const int64_t slot = static_cast<int64_t>(align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt)) /
                                            dtype_size(iter_dt));
  if (iter_dt == CSC_F32)
    hipLaunchKernelGGL(k_dir_moments<float>, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s,
                       static_cast<const float*>(basis), slot, nvec, m, part);
  else if (iter_half(iter_dt))
    hipLaunchKernelGGL(k_dir_moments<_Float16>, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s,
                       static_cast<const _Float16*>(basis), slot, nvec, m, part);
  else
    hipLaunchKernelGGL(k_dir_moments<uint16_t>, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, s,
                       static_cast<const uint16_t*>(basis), slot, nvec, m, part);
  hipLaunchKernelGGL(k_reduce_rows, dim3(m + 1), dim3(kThreads), 0, s, part, nb, moments);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace csc

// =====================================================================================
// Batched basis: the recurrences of S snapshots (same n, width and tile shape; each with its
// own graph, signals and basis) advance together, one launch per step.
namespace csc {

csc_status run_basis_batch(const Graph* const* graphs, int S, double lmax, int m,
                           const void* const* X, csc_dtype x_dt, int64_t ldx, int w,
                           csc_dtype iter_dt, int variant, void* const* bases, size_t bytes,
                           hipStream_t s, bool timed) {
  if (S < 1 || S > kMaxBatch) return fail(CSC_E_ARG, "batch size must be in [1, 8]");
  const int64_t n = graphs[0]->n;
  for (int i = 0; i < S; ++i) {
    if (graphs[i]->n != n) return fail(CSC_E_ARG, "batched graphs must have the same n");
    if (graphs[i]->val_dt != graphs[0]->val_dt) return fail(CSC_E_DTYPE, "batched graphs must share the value type");
  }
  if (m < 1 || w < 1 || ldx < w) return fail(CSC_E_ARG, "bad basis arguments");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "iterates must be F32, BF16, F16, BF16S or F16S");
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, 0);
  const size_t slot_bytes = align_up(static_cast<size_t>(n) * pl.wpad * dtype_size(iter_dt));
  const size_t state_bytes = align_up(static_cast<size_t>(n) * pl.wpad * state_size(iter_dt));
  if (bytes < basis_bytes(n, w, m, iter_dt, variant)) return fail(CSC_E_ARG, "basis buffer too small");
  const int wt = pl.shape.wt();
  auto state = [&](int i, int q) {
    return reinterpret_cast<float*>(static_cast<char*>(bases[i]) + static_cast<size_t>(m + 1) * slot_bytes +
                                    static_cast<size_t>(q) * state_bytes);
  };
  for (int i = 0; i < S; ++i)
    launch_init(iter_dt, X[i], x_dt, ldx, n, w, pl.wpad, wt, bases[i], nullptr, 0.f, state(i, 0), s);
  const BatchFn fn = batch_fn(iter_dt, pl.shape.lpr, graphs[0]->val_dt);
  const int64_t per = pl.row_blocks * pl.ntiles;
  double bytes_alg = 0.0;
  if (timed) timing_begin(s);
  for (int j = 0; j < m; ++j) {
    StepBatch b{};
    b.per = per;
    for (int i = 0; i < S; ++i) {
      StepParams& p = b.p[i];
      const Graph* g = graphs[i];
      char* base = static_cast<char*>(bases[i]);
      p.rowptr = g->rowptr;
      p.colidx = g->colidx;
      p.vals = g->vals;
      p.zcur = base + static_cast<size_t>(j) * slot_bytes;
      p.zprev = j > 0 ? base + static_cast<size_t>(j - 1) * slot_bytes : nullptr;
      p.zout = base + static_cast<size_t>(j + 1) * slot_bytes;
      p.scur = state(i, j & 1);
      p.sprev = state(i, (j + 1) & 1);
      p.sout = state(i, (j + 1) & 1);
      p.w = w;
      p.n = n;
      p.row_blocks = pl.row_blocks;
      const OpScale op = op_scale(g, lmax > 0.0 ? lmax : g->lmax_bound);
      set_op(p, op);
      p.flags = F_STORE | (j == 0 ? F_FIRST : 0) | (op.own() ? F_OWN : 0);
      bytes_alg += step_bytes(g, n, w, iter_dt, p.flags, CSC_F32);
    }
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(per * S)), dim3(kThreads), 0, s, b);
  }
  if (timed) timing_end(s, m, bytes_alg);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// S (<= 8) one-pass filters advanced together, one launch per step (the dynamic step's
// fresh blocks of several snapshots without kept iterates): snapshot i filters X[i] on
// graphs[i] with its own coefficients coefs[i][0..m] (device FP64, read by the kernels, so a
// captured sequence of launches stays valid when they change), accumulates in FP32 and
// stores Y[i] (y_dt) at the last step; with moments[i] != null it also returns the doubled
// moments mu_0..mu_m of X[i] (device).  work[i]: a filter workspace for (n, w, iter_dt) of
// least make_plan(n, w, iter_dt, variant, m).total bytes.
csc_status run_filter_batch(const Graph* const* graphs, int S, double lmax, int m,
                            const double* const* coefs, const void* const* X, csc_dtype x_dt,
                            int64_t ldx, void* const* Y, csc_dtype y_dt, int64_t ldy, int w,
                            csc_dtype iter_dt, int variant, double* const* moments,
                            void* const* work, size_t work_bytes, hipStream_t s, bool timed) {
  if (S < 1 || S > kMaxBatch) return fail(CSC_E_ARG, "batch size must be in [1, 8]");
  const int64_t n = graphs[0]->n;
  for (int i = 0; i < S; ++i) {
    if (graphs[i]->n != n) return fail(CSC_E_ARG, "batched graphs must have the same n");
    if (graphs[i]->val_dt != graphs[0]->val_dt) return fail(CSC_E_DTYPE, "batched graphs must share the value type");
  }
  if (m < 1 || w < 1 || ldx < w || ldy < w) return fail(CSC_E_ARG, "bad batched filter arguments");
  if (!iter_type_ok(iter_dt)) return fail(CSC_E_DTYPE, "iterates must be F32, BF16, F16, BF16S or F16S");
  const bool mom = moments != nullptr && moments[0] != nullptr;
  const FilterPlan pl = make_plan(n, w, iter_dt, variant, mom ? m : 0);
  if (work_bytes < pl.total) return fail(CSC_E_ARG, "batched filter workspace too small");
  const int wt = pl.shape.wt();
  auto at = [&](int i, size_t off) { return static_cast<char*>(work[i]) + off; };
  for (int i = 0; i < S; ++i)
    launch_init(iter_dt, X[i], x_dt, ldx, n, w, pl.wpad, wt, at(i, pl.off_z0),
                reinterpret_cast<float*>(at(i, pl.off_acc)), 0.f,
                reinterpret_cast<float*>(at(i, pl.off_s0)), s, coefs[i]);
  const BatchFn fn = batch_fn(iter_dt, pl.shape.lpr, graphs[0]->val_dt);
  const int64_t per = pl.row_blocks * pl.ntiles;
  const int J = m / 2;
  double bytes_alg = 0.0;
  if (timed) timing_begin(s);
  for (int j = 0; j < m; ++j) {
    StepBatch b{};
    b.per = per;
    const bool last = j == m - 1;
    for (int i = 0; i < S; ++i) {
      StepParams& p = b.p[i];
      const Graph* g = graphs[i];
      p.rowptr = g->rowptr;
      p.colidx = g->colidx;
      p.vals = g->vals;
      p.zcur = at(i, (j & 1) ? pl.off_z1 : pl.off_z0);
      p.zprev = at(i, (j & 1) ? pl.off_z0 : pl.off_z1);
      p.zout = at(i, (j & 1) ? pl.off_z0 : pl.off_z1);
      p.scur = reinterpret_cast<const float*>(at(i, (j & 1) ? pl.off_s1 : pl.off_s0));
      p.sprev = reinterpret_cast<const float*>(at(i, (j & 1) ? pl.off_s0 : pl.off_s1));
      p.sout = const_cast<float*>(p.sprev);
      p.acc = reinterpret_cast<float*>(at(i, pl.off_acc));
      p.ld_acc = pl.wpad;
      p.w = w;
      p.n = n;
      p.row_blocks = pl.row_blocks;
      const OpScale op = op_scale(g, lmax > 0.0 ? lmax : g->lmax_bound);
      set_op(p, op);
      p.coef_dev = coefs[i] + j + 1;
      int flags = F_ACC;
      if (j == 0) flags |= F_FIRST;
      if (last) {
        flags |= F_LAST;
        p.yout = Y[i];
        p.ldy = ldy;
        p.y_dt = int(y_dt);
      } else {
        flags |= F_STORE;
      }
      if (mom && j <= J) {
        flags |= F_MOM;
        p.mom_part = reinterpret_cast<double*>(at(i, pl.off_part)) + static_cast<int64_t>(j) * 2 * per;
      }
      if ((flags & F_MOM) || op.own()) flags |= F_OWN;
      p.flags = flags;
      bytes_alg += step_bytes(g, n, w, iter_dt, flags, y_dt);
    }
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(per * S)), dim3(kThreads), 0, s, b);
  }
  if (timed) timing_end(s, m, bytes_alg);
  CSC_HIP(hipGetLastError());
  if (mom) {
    for (int i = 0; i < S; ++i) {
      double* part = reinterpret_cast<double*>(at(i, pl.off_part));
      double* msum = reinterpret_cast<double*>(at(i, pl.off_mom));
      hipLaunchKernelGGL(k_reduce_rows, dim3(2 * (J + 1)), dim3(kThreads), 0, s, part, per, msum);
      hipLaunchKernelGGL(k_moments, dim3(1), dim3(64), 0, s, msum, J, m, moments[i]);
    }
    CSC_HIP(hipGetLastError());
  }
  return CSC_OK;
}

double filter_batch_bytes(const Graph* const* graphs, int S, int m, int w, csc_dtype iter_dt,
                          bool moments, csc_dtype y_dt) {
  double b = 0.0;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < m; ++j) {
      int flags = F_ACC | (j == 0 ? F_FIRST : 0) | (j == m - 1 ? F_LAST : F_STORE);
      if (moments && j <= m / 2) flags |= F_MOM | F_OWN;
      b += step_bytes(graphs[i], graphs[i]->n, w, iter_dt, flags, y_dt);
    }
  return b;
}

double basis_batch_bytes(const Graph* const* graphs, int S, int m, int w, csc_dtype iter_dt) {
  double b = 0.0;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < m; ++j)
      b += step_bytes(graphs[i], graphs[i]->n, w, iter_dt, F_STORE | (j == 0 ? F_FIRST : 0), CSC_F32);
  return b;
}

}  // namespace csc

// =====================================================================================
// Random-gather probe: the memory system's ceiling for the recurrence step's neighbour
// gathers.  For every row r of a CSR pattern, lane q of the row's group XORs the q-th 16-byte
// piece of the table rows named by the row's column indices, exactly the access pattern of
// the step kernel (CSR range staged in LDS, eight 16-byte loads in flight per lane, one row
// group of row_bytes / 16 lanes per row) with no arithmetic and no other stream.
namespace csc {

namespace {

template <int LPR>
__global__ __launch_bounds__(kThreads) void k_gather_probe(const int32_t* rowptr,
                                                           const int32_t* colidx, int64_t n,
                                                           const uint4* table, uint32_t* out) {
  constexpr int RPB = kThreads / LPR;
  __shared__ int32_t s_col[kStageCap];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RPB;
  const int64_t r1 = min(r0 + RPB, n);
  const int32_t e0 = rowptr[r0], e1 = rowptr[r1];
  const bool staged = e1 - e0 <= kStageCap;
  if (staged)
    for (int32_t i = threadIdx.x; i < e1 - e0; i += kThreads) s_col[i] = colidx[e0 + i];
  __syncthreads();
  const int64_t row = r0 + threadIdx.x / LPR;
  const int lane = threadIdx.x % LPR;
  if (row >= n) return;
  const int32_t rs = rowptr[row], re = rowptr[row + 1];
  const uint4* tb = table + lane;
  uint32_t acc = 0;
  int32_t e = rs;
  for (; e + 8 <= re; e += 8) {
    uint4 g[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t c = staged ? s_col[e + q - e0] : colidx[e + q];
      g[q] = tb[static_cast<int64_t>(c) * LPR];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc ^= g[q].x ^ g[q].y ^ g[q].z ^ g[q].w;
  }
  for (; e < re; ++e) {
    const int32_t c = staged ? s_col[e - e0] : colidx[e];
    const uint4 g = tb[static_cast<int64_t>(c) * LPR];
    acc ^= g.x ^ g.y ^ g.z ^ g.w;
  }
  out[row * LPR + lane] = acc;
}

}  // namespace

csc_status run_gather_probe(const int32_t* rowptr, const int32_t* colidx, int64_t n,
                            const void* table, int row_bytes, uint32_t* out, hipStream_t s) {
  if (n < 1 || !rowptr || !colidx || !table || !out) return fail(CSC_E_ARG, "bad probe arguments");
  const int64_t rpb = kThreads / (row_bytes / 16);
  const unsigned blocks = static_cast<unsigned>((n + rpb - 1) / rpb);
  const uint4* t = static_cast<const uint4*>(table);
  switch (row_bytes) {
    case 64: hipLaunchKernelGGL(k_gather_probe<4>, dim3(blocks), dim3(kThreads), 0, s, rowptr, colidx, n, t, out); break;
    case 128: hipLaunchKernelGGL(k_gather_probe<8>, dim3(blocks), dim3(kThreads), 0, s, rowptr, colidx, n, t, out); break;
    case 256: hipLaunchKernelGGL(k_gather_probe<16>, dim3(blocks), dim3(kThreads), 0, s, rowptr, colidx, n, t, out); break;
    case 512: hipLaunchKernelGGL(k_gather_probe<32>, dim3(blocks), dim3(kThreads), 0, s, rowptr, colidx, n, t, out); break;
    default: return fail(CSC_E_ARG, "row_bytes must be 64, 128, 256 or 512");
  }
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

}  // namespace csc
