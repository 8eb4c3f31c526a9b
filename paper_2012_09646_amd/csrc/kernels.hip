// Task kernels of the benchmark workloads, written for gfx950 (CDNA4):
// wave64, fp32 data in HBM, fp64 arithmetic in registers, one rounding to
// fp32 on store.  They are HBM-bound (coalesced float4 streams, LDS-tiled
// stencils, a merge-path CSR SpMV) and keep every reduction deterministic
// (fixed combination order, no floating-point atomics).  The one dense
// contraction, the ridge classifier's X W^T with C <= 16 classes, uses
// fp64 FMAs on the vector ALUs rather than MFMA: at C = 10 it does 5 flops
// per byte of X (below the fp64 ridge point of ~10 flops/byte), gfx950's
// fp64 MFMA peak is no higher than its fp64 vector peak, and a 16-wide MFMA
// tile would waste 6 of 16 columns.
//
// Benchmarks (paper Sec. V-B): VEC sums the difference of two squared
// vectors; B&S prices European calls in double precision; IMG combines a
// sharpened image with blurred copies; HITS repeats SpMV with a matrix and
// its transpose; ML averages the posteriors of two classifiers.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/dagrt.h"
#include "kernels.hpp"

namespace dagrt {
namespace {

// Timing of a task's kernels: when set, the first dispatch of the task takes
// the start event and every dispatch the stop event (the last one wins), both
// attached to the dispatch packets themselves.
thread_local hipEvent_t tl_start = nullptr;
thread_local hipEvent_t tl_stop = nullptr;

#define DAGRT_LAUNCH(kern, grid, block, shmem, stream, ...)                                       \
  do {                                                                                            \
    if (tl_stop) {                                                                                \
      hipEvent_t st_ = tl_start;                                                                  \
      tl_start = nullptr;                                                                         \
      hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, st_, tl_stop, 0, __VA_ARGS__);      \
    } else {                                                                                      \
      hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                          \
    }                                                                                             \
  } while (0)

constexpr int kWave = 64;
uint64_t g_wall_khz = 100000;  // device constant-rate clock (kHz)

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// ---------------------------------------------------------------------------
// Wave / workgroup reductions (butterfly: every lane ends with the same value)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum over the workgroup (<= 1024 threads); every thread gets the result.
__device__ double block_sum(double v, double* sh /* 17 entries */) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    double r = lane < nw ? sh[lane] : 0.0;
    r = wave_sum(r);
    if (lane == 0) sh[16] = r;
  }
  __syncthreads();
  const double r = sh[16];
  __syncthreads();
  return r;
}

__device__ void block_minmax(float* mx, float* mn, float* sh /* 34 entries */) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  float a = wave_max(*mx), b = wave_min(*mn);
  if (lane == 0) {
    sh[w] = a;
    sh[16 + w] = b;
  }
  __syncthreads();
  if (w == 0) {
    a = lane < nw ? sh[lane] : -INFINITY;
    b = lane < nw ? sh[16 + lane] : INFINITY;
    a = wave_max(a);
    b = wave_min(b);
    if (lane == 0) {
      sh[32] = a;
      sh[33] = b;
    }
  }
  __syncthreads();
  *mx = sh[32];
  *mn = sh[33];
  __syncthreads();
}

// Grid-wide completion: each workgroup publishes its partial, then takes a
// ticket; the workgroup holding the last ticket combines all partials in
// index order.  Agent-scope release/acquire makes the partials visible
// across XCDs (each has its own L2).
__device__ __forceinline__ void publish_partial(uint64_t* partials, uint64_t bits) {
  if (threadIdx.x == 0)
    __hip_atomic_store(&partials[blockIdx.x], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t read_partial(const uint64_t* partials, uint32_t i) {
  return __hip_atomic_load(const_cast<uint64_t*>(partials) + i, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ bool arrive_last(uint32_t* counter, int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}
__device__ __forceinline__ void reset_counter(uint32_t* counter) {
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t d2u(double d) { return static_cast<uint64_t>(__double_as_longlong(d)); }
__device__ __forceinline__ double u2d(uint64_t u) { return __longlong_as_double(static_cast<long long>(u)); }

// ---------------------------------------------------------------------------
// VEC: x <- x*x (one fp32 product, bit-exact with IEEE single precision)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_vec_square(float* __restrict__ x, uint64_t n, int vec) {
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  if (vec) {
    float4* x4 = reinterpret_cast<float4*>(x);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      float4 v = x4[i];
      v.x *= v.x;
      v.y *= v.y;
      v.z *= v.z;
      v.w *= v.w;
      x4[i] = v;
    }
    for (uint64_t i = (n4 << 2) + gid; i < n; i += stride) x[i] *= x[i];
  } else {
    for (uint64_t i = gid; i < n; i += stride) x[i] *= x[i];
  }
}

// Two ways to combine the per-workgroup partials, chosen by the launch
// variant: 0 = a second one-workgroup kernel sums them (the kernel boundary
// makes them visible); 1 = single pass, the last workgroup to arrive sums
// them (one agent-scope release per workgroup: each XCD has its own L2).

// r[0] = fl32(sum_i (x_i - y_i)) with fp64 differences and accumulation.
template <bool kSinglePass>
__global__ __launch_bounds__(1024) void k_vec_sum_diff(const float* __restrict__ x,
                                                       const float* __restrict__ y,
                                                       float* __restrict__ r, uint64_t n, int vec,
                                                       uint32_t* counter, uint64_t* partials) {
  __shared__ double sh[17];
  __shared__ int flag;
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  double acc = 0.0;
  if (vec) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 a = x4[i], b = y4[i];
      acc += static_cast<double>(a.x) - static_cast<double>(b.x);
      acc += static_cast<double>(a.y) - static_cast<double>(b.y);
      acc += static_cast<double>(a.z) - static_cast<double>(b.z);
      acc += static_cast<double>(a.w) - static_cast<double>(b.w);
    }
    for (uint64_t i = (n4 << 2) + gid; i < n; i += stride)
      acc += static_cast<double>(x[i]) - static_cast<double>(y[i]);
  } else {
    for (uint64_t i = gid; i < n; i += stride)
      acc += static_cast<double>(x[i]) - static_cast<double>(y[i]);
  }
  const double bsum = block_sum(acc, sh);
  publish_partial(partials, d2u(bsum));
  if (kSinglePass && arrive_last(counter, &flag)) {
    double t = 0.0;
    for (uint32_t i = threadIdx.x; i < gridDim.x; i += blockDim.x) t += u2d(read_partial(partials, i));
    const double tot = block_sum(t, sh);
    if (threadIdx.x == 0) r[0] = static_cast<float>(tot);
    reset_counter(counter);
  }
}

// Second pass: one workgroup sums np fp64 partials in a fixed order.
template <typename Out>
__global__ __launch_bounds__(256) void k_finish_sum(const uint64_t* __restrict__ partials, uint32_t np,
                                                    Out* __restrict__ out) {
  __shared__ double sh[17];
  double t = 0.0;
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) t += u2d(partials[i]);
  const double tot = block_sum(t, sh);
  if (threadIdx.x == 0) out[0] = static_cast<Out>(tot);
}

// ---------------------------------------------------------------------------
// B&S: European call, C = S N(d1) - K e^{-rT} N(d2), N(z) = erfc(-z/sqrt2)/2
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bs_price(double s, double strike, double mu_t, double vol_t,
                                           double disc_strike) {
  const double d1 = (log(s / strike) + mu_t) / vol_t;
  const double d2 = d1 - vol_t;
  const double n1 = 0.5 * erfc(-d1 * M_SQRT1_2);
  const double n2 = 0.5 * erfc(-d2 * M_SQRT1_2);
  return s * n1 - disc_strike * n2;
}

// Per-launch constants of the call price.
struct BsConst {
  double strike, mu_t, vol_t, disc_strike;  // K, (r + vol^2/2) T, vol sqrt(T), K e^{-rT}
  double inv_strike, inv_vol_t, growth;     // 1/K, 1/(vol sqrt(T)), e^{rT}/K
};

#include "erfcx_poly.inc"

// erfcx(a) = exp(a^2) erfc(a) for a >= 0 from one polynomial in
// y = 2t - 1, t = K/(K + a) (coefficients fitted offline to 1.8e-15).
__device__ __forceinline__ double erfcx_pos(double a) {
  // t by the hardware reciprocal and two Newton steps (error below 1 ulp of
  // the fit's accuracy; the divisor is >= K, so no denormal or zero cases)
  const double x = kErfcxK + a;
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  const double t = kErfcxK * r;
  const double y = 2.0 * t - 1.0;
  double g = kErfcxC[kErfcxDegree];
#pragma unroll
  for (int k = kErfcxDegree - 1; k >= 0; --k) g = fma(g, y, kErfcxC[k]);
  return t * g;
}

// Same price with one exponential per option: N(d) = h or 1 - h with
// h = exp(-d^2/2) erfcx(|d|/sqrt2)/2, and exp(-d2^2/2) = exp(-d1^2/2) S e^{rT}/K
// (d1^2 - d2^2 = 2 (ln(S/K) + rT)).  Where exp(-d1^2/2) underflows the second
// exponential is computed directly.
__device__ __forceinline__ double bs_price_fast(double s, const BsConst& k) {
  const double d1 = (log(s * k.inv_strike) + k.mu_t) * k.inv_vol_t;
  const double d2 = d1 - k.vol_t;
  const double e1 = exp(-0.5 * d1 * d1);
  double e2 = e1 * s * k.growth;
  if (e1 == 0.0) e2 = exp(-0.5 * d2 * d2);
  const double h1 = 0.5 * e1 * erfcx_pos(fabs(d1) * M_SQRT1_2);
  const double h2 = 0.5 * e2 * erfcx_pos(fabs(d2) * M_SQRT1_2);
  const double n1 = d1 < 0.0 ? h1 : 1.0 - h1;
  const double n2 = d2 < 0.0 ? h2 : 1.0 - h2;
  // a zero spot prices at 0 (ln 0 = -inf would reach erfcx_pos(inf) = NaN);
  // spots must not be negative (the model's domain)
  const double c = s * n1 - k.disc_strike * n2;
  return s > 0.0 ? c : 0.0;
}

// a * b + c as one three-address v_fma_f64.  For a Horner step whose
// coefficient sits in a vector register (the kernel keeps more constants than
// the scalar registers hold), the compiler otherwise picks the accumulating
// form, which overwrites its addend, and copies the coefficient first: one
// extra 64-bit move per step.
__device__ __forceinline__ double fma_3addr(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// ln 2 split so that k * kLn2Hi is exact for |k| < 2^21 (its low 21 mantissa
// bits are zero); kLn2Lo is the rest.
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;

// e^x for x <= 0 without special-case handling: x = k ln2 + r, |r| <= ln2/2,
// e^r by its Taylor series to r^13 (next term below 5e-18), scaled by 2^k.
// Below -746 the result is 0 (clamped so k stays a small integer).
__device__ __forceinline__ double exp_nonpos(double x) {
  x = fmax(x, -746.0);
  const double kd = rint(x * 0x1.71547652b82fep+0);  // x log2(e)
  double r = fma(-kd, kLn2Hi, x);
  r = fma(-kd, kLn2Lo, r);
  constexpr double c[14] = {0x1.0p+0, 0x1.0p+0, 0x1.0p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5,
                            0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
                            0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22,
                            0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};  // 1/n!
  double p = c[13];
#pragma unroll
  for (int i = 12; i >= 0; --i) p = fma_3addr(p, r, c[i]);
  return ldexp(p, static_cast<int>(kd));
}

// ln y for finite y > 0 in the normal range: y = m 2^e with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(u), u = (m - 1)/(m + 1), |u| <= 0.172,
// by its series to u^19 (next term below 5e-18); u by the hardware
// reciprocal and two Newton steps.
__device__ __forceinline__ double log_pos(double y) {
  int e;
  double m = frexp(y, &e);  // m in [0.5, 1)
  if (m < M_SQRT1_2) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;  // exact
  const double x = 2.0 + f;
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  const double u = f * r, u2 = u * u;
  constexpr double c[10] = {0x1.0p+0, 0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
                            0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
                            0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5};  // 1/(2n+1)
  double q = c[9];
#pragma unroll
  for (int i = 8; i >= 0; --i) q = fma_3addr(q, u2, c[i]);
  const double ed = static_cast<double>(e);
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, 2.0 * u * q));
}

// bs_price_fast with the exponential and logarithm above (inputs there are
// finite: S * (1/K) is a normal double for every positive fp32 S, the
// exponent is -d^2/2 <= 0).  A zero spot prices at 0 (the limit of the
// formula); log_pos(0) is not -inf, so that is selected at the end, as in
// bs_price_fast (one compare and select).  Spots must not be negative.
__device__ __forceinline__ double bs_price_own(double s, const BsConst& k) {
  const double d1 = (log_pos(s * k.inv_strike) + k.mu_t) * k.inv_vol_t;
  const double d2 = d1 - k.vol_t;
  const double e1 = exp_nonpos(-0.5 * d1 * d1);
  double e2 = e1 * s * k.growth;
  if (e1 == 0.0) e2 = exp_nonpos(-0.5 * d2 * d2);
  const double h1 = 0.5 * e1 * erfcx_pos(fabs(d1) * M_SQRT1_2);
  const double h2 = 0.5 * e2 * erfcx_pos(fabs(d2) * M_SQRT1_2);
  const double n1 = d1 < 0.0 ? h1 : 1.0 - h1;
  const double n2 = d2 < 0.0 ? h2 : 1.0 - h2;
  const double c = s * n1 - k.disc_strike * n2;
  return s > 0.0 ? c : 0.0;
}

// variant 0: the library's erfc; 1: bs_price_fast; 2: bs_price_own.
template <int V>
__device__ __forceinline__ float bs_one(float s, const BsConst& k) {
  if constexpr (V == 0) {
    return static_cast<float>(bs_price(s, k.strike, k.mu_t, k.vol_t, k.disc_strike));
  } else if constexpr (V == 1) {
    return static_cast<float>(bs_price_fast(s, k));
  } else {
    return static_cast<float>(bs_price_own(s, k));
  }
}

template <int V>
__global__ __launch_bounds__(1024) void k_bs_call(const float* __restrict__ S, float* __restrict__ C,
                                                  uint64_t n, int vec, BsConst k) {
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  if (vec) {
    const float4* s4 = reinterpret_cast<const float4*>(S);
    float4* c4 = reinterpret_cast<float4*>(C);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 s = s4[i];
      float4 c;
      c.x = bs_one<V>(s.x, k);
      c.y = bs_one<V>(s.y, k);
      c.z = bs_one<V>(s.z, k);
      c.w = bs_one<V>(s.w, k);
      c4[i] = c;
    }
    for (uint64_t i = (n4 << 2) + gid; i < n; i += stride) C[i] = bs_one<V>(S[i], k);
  } else {
    for (uint64_t i = gid; i < n; i += stride) C[i] = bs_one<V>(S[i], k);
  }
}

// ---------------------------------------------------------------------------
// IMG: LDS-tiled stencils with clamp-to-edge borders.  A workgroup produces a
// TW x TH output tile with TW * TH / 4 threads, each thread four rows of one
// column.  Tile shapes (launch variant >> 1): 64 x 16 (256 threads, the
// default), 64 x 8 (128), 64 x 4 (64) and 32 x 8 (64).
// ---------------------------------------------------------------------------
constexpr int kRowsPerThread = 4;

struct GaussW {
  double w[31];
};

// Tile of this workgroup (1-D grid).  xcd_map = 0: tile = block id, row-major.
// xcd_map = 1: the dispatcher hands workgroups to the 8 XCDs round-robin by
// id, so block b runs on XCD b % 8; giving each XCD one contiguous run of
// row-major tiles keeps a tile and its left, right, upper and lower
// neighbours, whose halos overlap it, on one XCD and so in one L2.  Returns
// false for the padding blocks of the last run (uniform per workgroup).
template <int TW, int TH>
__device__ __forceinline__ bool tile_of(int tiles_x, int ntiles, int xcd_map, int* x0, int* y0) {
  int t = blockIdx.x;
  if (xcd_map) {
    const int per = (ntiles + 7) / 8;
    t = static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8);
    if (t >= ntiles) return false;
  }
  *x0 = (t % tiles_x) * TW;
  *y0 = (t / tiles_x) * TH;
  return true;
}

// Stage image rows [y0 - R, y0 - R + IH) x columns [x0 - R, x0 - R + TW + 2R)
// (clamped to the border) into s.  64-wide tiles: a lane keeps one column for
// the whole tile and each wave takes every NT/64-th row, so the row is uniform
// per wave and a load costs an add; the 2R halo columns are a second load by
// the first 2R lanes.  Other widths: the threads stride over the tile.
template <int R, int TW, int IH, int SW, int NT>
__device__ __forceinline__ void stage_tile(const float* __restrict__ in, float (*s)[SW], int w, int h, int x0,
                                           int y0) {
  static_assert(SW >= TW + 2 * R, "LDS row too narrow");
  if constexpr (TW == 64 && NT % 64 == 0 && 2 * R <= 64) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gx_main = min(max(x0 - R + lane, 0), w - 1);
    const int gx_halo = min(max(x0 - R + TW + lane, 0), w - 1);
#pragma unroll
    for (int k = 0; k < (IH + NW - 1) / NW; ++k) {
      const int r = wv + NW * k;
      if (r < IH) {
        const int gy = min(max(y0 - R + r, 0), h - 1);
        const float* row = in + static_cast<size_t>(gy) * w;
        s[r][lane] = row[gx_main];
        if (lane < 2 * R) s[r][TW + lane] = row[gx_halo];
      }
    }
  } else {
    constexpr int IW = TW + 2 * R;
    for (int idx = threadIdx.x; idx < IH * IW; idx += NT) {
      const int r = idx / IW, c = idx - r * IW;
      const int gy = min(max(y0 - R + r, 0), h - 1);
      const int gx = min(max(x0 - R + c, 0), w - 1);
      s[r][c] = in[static_cast<size_t>(gy) * w + gx];
    }
  }
}

// A 64-wide tile's rows with their halo held in registers: the same lane and
// row assignment as stage_tile's 64-wide path (lane = column, wave = every
// NW-th row), so that the loads of the next tile can be in flight while the
// current one is computed from LDS.
template <int R, int TH, int NT>
struct TileRows {
  static constexpr int NW = NT / 64;
  static constexpr int IH = TH + 2 * R;
  static constexpr int RPW = (IH + NW - 1) / NW;
  static_assert(NT % 64 == 0 && 2 * R <= 64, "64-wide tiles with at most 64 halo columns");
  float m[RPW];
  float hl[RPW];
  __device__ __forceinline__ void load(const float* __restrict__ in, int w, int h, int x0, int y0) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gx_main = min(max(x0 - R + lane, 0), w - 1);
    const int gx_halo = min(max(x0 - R + 64 + lane, 0), w - 1);
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = wv + NW * k;
      if (r < IH) {
        const float* row = in + static_cast<size_t>(min(max(y0 - R + r, 0), h - 1)) * w;
        m[k] = row[gx_main];
        if (lane < 2 * R) hl[k] = row[gx_halo];
      }
    }
  }
  template <int SW>
  __device__ __forceinline__ void store(float (*s)[SW]) const {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = wv + NW * k;
      if (r < IH) {
        s[r][lane] = m[k];
        if (lane < 2 * R) s[r][64 + lane] = hl[k];
      }
    }
  }
};

// Resident grid over 64-wide tiles: gridDim.x is a multiple of 8 and block b
// runs on XCD b % 8, which walks its contiguous run of row-major tiles (as in
// tile_of's xcd_map = 1) with gridDim.x / 8 workgroups side by side.
struct ResidentTiles {
  int t, end, step;
  __device__ __forceinline__ explicit ResidentTiles(int ntiles) {
    const int per = (ntiles + 7) / 8;
    const int xcd = static_cast<int>(blockIdx.x % 8);
    t = xcd * per + static_cast<int>(blockIdx.x / 8);
    end = min(ntiles, (xcd + 1) * per);
    step = static_cast<int>(gridDim.x / 8);
  }
};

// The blur's two passes over a staged tile: horizontal into the fp64 tile
// s_h, barrier, vertical to the output.
template <int R, int TW, int TH>
__device__ __forceinline__ void blur_passes(const float (*s_in)[TW + 2 * R], double (*s_h)[TW],
                                            float* __restrict__ out, int w, int h, const GaussW& wt, int x0,
                                            int y0) {
  constexpr int G = kRowsPerThread;
  constexpr int NT = TW * TH / G;
  constexpr int K = 2 * R + 1;
  constexpr int IH = TH + 2 * R;
  // horizontal pass: each work item produces 4 adjacent outputs of one row
  // from one register window of 4 + 2R inputs (4x fewer LDS reads)
  for (int item = threadIdx.x; item < IH * (TW / G); item += NT) {
    const int r = item / (TW / G), c0 = (item % (TW / G)) * G;
    float v[G + 2 * R];
#pragma unroll
    for (int j = 0; j < G + 2 * R; ++j) v[j] = s_in[r][c0 + j];
#pragma unroll
    for (int o = 0; o < G; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) acc += wt.w[j] * static_cast<double>(v[o + j]);
      s_h[r][c0 + o] = acc;
    }
  }
  __syncthreads();
  // vertical pass: each thread produces 4 rows of one column from one window
  const int c = threadIdx.x % TW;
  const int r0 = (threadIdx.x / TW) * G;
  const int gx = x0 + c;
  double v[G + 2 * R];
#pragma unroll
  for (int j = 0; j < G + 2 * R; ++j) v[j] = s_h[r0 + j][c];
#pragma unroll
  for (int o = 0; o < G; ++o) {
    const int gy = y0 + r0 + o;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) acc += wt.w[i] * v[o + i];
    if (gx < w && gy < h) out[static_cast<size_t>(gy) * w + gx] = static_cast<float>(acc);
  }
}

// Separable Gaussian: stage the input tile with its halo in LDS (fp32, as
// stored), horizontal pass into an fp64 LDS tile, vertical pass to output.
template <int R, int TW, int TH>
__global__ __launch_bounds__(TW * TH / kRowsPerThread) void k_gauss_blur(const float* __restrict__ in,
                                                                          float* __restrict__ out, int w, int h,
                                                                          GaussW wt, int tiles_x, int ntiles,
                                                                          int xcd_map) {
  constexpr int NT = TW * TH / kRowsPerThread;
  constexpr int IW = TW + 2 * R;
  constexpr int IH = TH + 2 * R;
  __shared__ float s_in[IH][IW];
  __shared__ double s_h[IH][TW];
  int x0, y0;
  if (!tile_of<TW, TH>(tiles_x, ntiles, xcd_map, &x0, &y0)) return;
  stage_tile<R, TW, IH, IW, NT>(in, s_in, w, h, x0, y0);
  __syncthreads();
  blur_passes<R, TW, TH>(s_in, s_h, out, w, h, wt, x0, y0);
}

// The same blur on a resident grid (64-wide tiles): each workgroup walks its
// XCD's tiles, holding the next tile's rows in registers while it computes
// the current one, so that the loads overlap the arithmetic.
template <int R, int TH>
__global__ __launch_bounds__(64 * TH / kRowsPerThread) void k_gauss_blur_rt(const float* __restrict__ in,
                                                                             float* __restrict__ out, int w, int h,
                                                                             GaussW wt, int tiles_x, int ntiles) {
  constexpr int TW = 64;
  constexpr int NT = TW * TH / kRowsPerThread;
  constexpr int IH = TH + 2 * R;
  __shared__ float s_in[IH][TW + 2 * R];
  __shared__ double s_h[IH][TW];
  ResidentTiles it(ntiles);
  TileRows<R, TH, NT> next;
  if (it.t < it.end) next.load(in, w, h, (it.t % tiles_x) * TW, (it.t / tiles_x) * TH);
  for (; it.t < it.end; it.t += it.step) {  // uniform per workgroup
    const int x0 = (it.t % tiles_x) * TW, y0 = (it.t / tiles_x) * TH;
    // every thread left the previous tile's horizontal pass (the barrier in
    // blur_passes) before any writes s_in, and its vertical pass before the
    // barrier below, after which s_h is written again
    next.store(s_in);
    __syncthreads();
    const int tn = it.t + it.step;
    if (tn < it.end) next.load(in, w, h, (tn % tiles_x) * TW, (tn / tiles_x) * TH);
    blur_passes<R, TW, TH>(s_in, s_h, out, w, h, wt, x0, y0);
  }
}

// Sobel gradient magnitude sqrt(gx^2 + gy^2), gx with [[-1,0,1],[-2,0,2],
// [-1,0,1]] (correlation), gy with its transpose, over a staged tile.
template <int TW, int TH>
__device__ __forceinline__ void sobel_tile(const float (*s_in)[TW + 2], float* __restrict__ out, int w, int h,
                                           int x0, int y0) {
  constexpr int G = kRowsPerThread;
  // each thread: 4 rows of one column from a 6 x 3 register window
  const int c = threadIdx.x % TW;
  const int r0 = (threadIdx.x / TW) * G;
  const int gx = x0 + c;
  double p[G + 2][3];
#pragma unroll
  for (int j = 0; j < G + 2; ++j) {
    p[j][0] = s_in[r0 + j][c];
    p[j][1] = s_in[r0 + j][c + 1];
    p[j][2] = s_in[r0 + j][c + 2];
  }
#pragma unroll
  for (int o = 0; o < G; ++o) {
    const int gy = y0 + r0 + o;
    const double sx = (p[o][2] - p[o][0]) + 2.0 * (p[o + 1][2] - p[o + 1][0]) + (p[o + 2][2] - p[o + 2][0]);
    const double sy = (p[o + 2][0] - p[o][0]) + 2.0 * (p[o + 2][1] - p[o][1]) + (p[o + 2][2] - p[o][2]);
    if (gx < w && gy < h) out[static_cast<size_t>(gy) * w + gx] = static_cast<float>(sqrt(sx * sx + sy * sy));
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH / kRowsPerThread) void k_sobel(const float* __restrict__ in,
                                                                     float* __restrict__ out, int w, int h,
                                                                     int tiles_x, int ntiles, int xcd_map) {
  constexpr int NT = TW * TH / kRowsPerThread;
  constexpr int IW = TW + 2, IH = TH + 2;
  __shared__ float s_in[IH][IW];
  int x0, y0;
  if (!tile_of<TW, TH>(tiles_x, ntiles, xcd_map, &x0, &y0)) return;
  stage_tile<1, TW, IH, IW, NT>(in, s_in, w, h, x0, y0);
  __syncthreads();
  sobel_tile<TW, TH>(s_in, out, w, h, x0, y0);
}

// Sobel on a resident grid of 64-wide tiles, the next tile's rows loaded
// into registers during the current tile's arithmetic (as k_gauss_blur_rt).
template <int TH>
__global__ __launch_bounds__(64 * TH / kRowsPerThread) void k_sobel_rt(const float* __restrict__ in,
                                                                        float* __restrict__ out, int w, int h,
                                                                        int tiles_x, int ntiles) {
  constexpr int TW = 64;
  constexpr int NT = TW * TH / kRowsPerThread;
  __shared__ float s_in[TH + 2][TW + 2];
  ResidentTiles it(ntiles);
  TileRows<1, TH, NT> next;
  if (it.t < it.end) next.load(in, w, h, (it.t % tiles_x) * TW, (it.t / tiles_x) * TH);
  for (; it.t < it.end; it.t += it.step) {  // uniform per workgroup
    const int x0 = (it.t % tiles_x) * TW, y0 = (it.t / tiles_x) * TH;
    next.store(s_in);
    __syncthreads();
    const int tn = it.t + it.step;
    if (tn < it.end) next.load(in, w, h, (tn % tiles_x) * TW, (tn / tiles_x) * TH);
    sobel_tile<TW, TH>(s_in, out, w, h, x0, y0);
    __syncthreads();  // every read of s_in done before the next tile's rows overwrite it
  }
}

// M = [max, min] of n fp32 values (exact).
template <bool kSinglePass>
__global__ __launch_bounds__(1024) void k_minmax(const float* __restrict__ a, float* __restrict__ M,
                                                 uint64_t n, int vec, uint32_t* counter,
                                                 uint64_t* partials) {
  __shared__ float sh[34];
  __shared__ int flag;
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  float mx = -INFINITY, mn = INFINITY;
  if (vec) {
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 v = a4[i];
      mx = fmaxf(mx, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
      mn = fminf(mn, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
    }
    for (uint64_t i = (n4 << 2) + gid; i < n; i += stride) {
      mx = fmaxf(mx, a[i]);
      mn = fminf(mn, a[i]);
    }
  } else {
    for (uint64_t i = gid; i < n; i += stride) {
      mx = fmaxf(mx, a[i]);
      mn = fminf(mn, a[i]);
    }
  }
  block_minmax(&mx, &mn, sh);
  publish_partial(partials, (static_cast<uint64_t>(__float_as_uint(mx)) << 32) | __float_as_uint(mn));
  if (kSinglePass && arrive_last(counter, &flag)) {
    float gmx = -INFINITY, gmn = INFINITY;
    for (uint32_t i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
      const uint64_t u = read_partial(partials, i);
      gmx = fmaxf(gmx, __uint_as_float(static_cast<uint32_t>(u >> 32)));
      gmn = fminf(gmn, __uint_as_float(static_cast<uint32_t>(u & 0xffffffffu)));
    }
    block_minmax(&gmx, &gmn, sh);
    if (threadIdx.x == 0) {
      M[0] = gmx;
      M[1] = gmn;
    }
    reset_counter(counter);
  }
}

__global__ __launch_bounds__(256) void k_finish_minmax(const uint64_t* __restrict__ partials, uint32_t np,
                                                       float* __restrict__ M) {
  __shared__ float sh[34];
  float gmx = -INFINITY, gmn = INFINITY;
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) {
    const uint64_t u = partials[i];
    gmx = fmaxf(gmx, __uint_as_float(static_cast<uint32_t>(u >> 32)));
    gmn = fminf(gmn, __uint_as_float(static_cast<uint32_t>(u & 0xffffffffu)));
  }
  block_minmax(&gmx, &gmn, sh);
  if (threadIdx.x == 0) {
    M[0] = gmx;
    M[1] = gmn;
  }
}

// N = (S - min) / (max - min) in fp64; all zeros when max == min.
__device__ __forceinline__ float norm1(float s, double mn, double d) {
  return d == 0.0 ? 0.0f : static_cast<float>((static_cast<double>(s) - mn) / d);
}
__global__ __launch_bounds__(1024) void k_normalise(const float* __restrict__ S,
                                                    const float* __restrict__ M,
                                                    float* __restrict__ N, uint64_t n, int vec) {
  const double mx = M[0], mn = M[1];
  const double d = mx - mn;
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  if (vec) {
    const float4* s4 = reinterpret_cast<const float4*>(S);
    float4* o4 = reinterpret_cast<float4*>(N);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 s = s4[i];
      o4[i] = make_float4(norm1(s.x, mn, d), norm1(s.y, mn, d), norm1(s.z, mn, d), norm1(s.w, mn, d));
    }
    for (uint64_t i = (n4 << 2) + gid; i < n; i += stride) N[i] = norm1(S[i], mn, d);
  } else {
    for (uint64_t i = gid; i < n; i += stride) N[i] = norm1(S[i], mn, d);
  }
}

// Unsharp-mask combine: E = (N3+N7+N15)/3, sharp = 2 img - B3,
// soft = (B7+B15)/2, out = clamp(E sharp + (1-E) soft, 0, 1).
__device__ __forceinline__ float combine1(float img, float b3, float b7, float b15, float n3,
                                          float n7, float n15) {
  const double e = (static_cast<double>(n3) + static_cast<double>(n7) + static_cast<double>(n15)) / 3.0;
  const double sharp = 2.0 * static_cast<double>(img) - static_cast<double>(b3);
  const double soft = 0.5 * (static_cast<double>(b7) + static_cast<double>(b15));
  const double o = e * sharp + (1.0 - e) * soft;
  return static_cast<float>(fmin(fmax(o, 0.0), 1.0));
}
__global__ __launch_bounds__(1024) void k_unsharp_combine(
    const float* __restrict__ img, const float* __restrict__ b3, const float* __restrict__ b7,
    const float* __restrict__ b15, const float* __restrict__ n3, const float* __restrict__ n7,
    const float* __restrict__ n15, float* __restrict__ out, uint64_t n, int vec) {
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t start = 0;
  if (vec) {
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 a = reinterpret_cast<const float4*>(img)[i];
      const float4 p = reinterpret_cast<const float4*>(b3)[i];
      const float4 q = reinterpret_cast<const float4*>(b7)[i];
      const float4 u = reinterpret_cast<const float4*>(b15)[i];
      const float4 e3 = reinterpret_cast<const float4*>(n3)[i];
      const float4 e7 = reinterpret_cast<const float4*>(n7)[i];
      const float4 e15 = reinterpret_cast<const float4*>(n15)[i];
      reinterpret_cast<float4*>(out)[i] =
          make_float4(combine1(a.x, p.x, q.x, u.x, e3.x, e7.x, e15.x),
                      combine1(a.y, p.y, q.y, u.y, e3.y, e7.y, e15.y),
                      combine1(a.z, p.z, q.z, u.z, e3.z, e7.z, e15.z),
                      combine1(a.w, p.w, q.w, u.w, e3.w, e7.w, e15.w));
    }
    start = n4 << 2;
  }
  for (uint64_t i = start + gid; i < n; i += stride)
    out[i] = combine1(img[i], b3[i], b7[i], b15[i], n3[i], n7[i], n15[i]);
}

// ---------------------------------------------------------------------------
// HITS: CSR SpMV (merge-path over row ends and nonzeros, so a row with
// millions of nonzeros is split evenly across workgroups), sum of squares,
// L2 scaling.
// ---------------------------------------------------------------------------
struct SpmvScratch {
  int* coord;         // per tile boundary b (0..ntiles): rows finished before diagonal b*TILE
  int* head_row;      // per tile: row whose sum continues from earlier tiles, or -1
  int* tail_row;      // per tile: row open at the end of the tile
  double* head_val;   // per tile: this tile's part of head_row (incl. in-tile carry)
  double* tail_val;   // per tile: this tile's part of tail_row
};

__device__ __forceinline__ int clamp_nnz(int v, int nnz) { return min(max(v, 0), nnz); }

// Merge-path split of diagonal `diag` (rows finished before it) by one wave:
// the smallest x in [max(0, diag - nnz), min(diag, nrows)] whose row end is
// past diag - x - 1.  64 probes per round shrink the interval 65-fold, so a
// few dependent global loads replace a long binary-search chain.
__device__ long long wave_merge_search(const int* __restrict__ row_ptr, int nrows, int nnz,
                                       long long diag) {
  const int lane = threadIdx.x & (kWave - 1);
  long long lo = max(0LL, diag - nnz), hi = min(diag, static_cast<long long>(nrows));
  while (hi - lo > kWave) {
    const long long span = hi - lo;
    const long long x = lo + ((lane + 1) * span) / (kWave + 1);
    const bool p = clamp_nnz(row_ptr[x + 1], nnz) <= diag - x - 1;
    const int c = __popcll(__ballot(p));
    if (c == 0) {
      hi = lo + span / (kWave + 1);
    } else {
      const long long sc1 = lo + (static_cast<long long>(c) * span) / (kWave + 1);
      const long long nhi = c < kWave ? lo + ((c + 1) * span) / (kWave + 1) : hi;
      lo = sc1 + 1;
      hi = nhi;
    }
  }
  const long long x = lo + lane;
  const bool p = x < hi && clamp_nnz(row_ptr[x + 1], nnz) <= diag - x - 1;
  return lo + __popcll(__ballot(p));
}

// Tile boundaries of the merge path, one wave per boundary, all in parallel.
__global__ __launch_bounds__(256) void k_spmv_partition(const int* __restrict__ row_ptr, int nrows,
                                                        int nnz, int tile, int ntiles, SpmvScratch sc) {
  const int b = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (b > ntiles) return;
  const long long total = static_cast<long long>(nrows) + nnz;
  const long long diag = min(static_cast<long long>(b) * tile, total);
  const long long x = wave_merge_search(row_ptr, nrows, nnz, diag);
  if ((threadIdx.x & (kWave - 1)) == 0) sc.coord[b] = static_cast<int>(x);
}

template <int IPT>
__global__ __launch_bounds__(256) void k_spmv_merge(const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const float* __restrict__ x,
                                                    float* __restrict__ y, int nrows, int ncols,
                                                    int nnz, SpmvScratch sc) {
  constexpr int TILE = 256 * IPT;
  __shared__ int s_rowend[TILE + 1];
  __shared__ double s_prod[TILE];
  __shared__ float s_out[TILE];  // rows finished in this tile, written out coalesced
  __shared__ int s_wrow[256 / kWave];
  __shared__ double s_wsum[256 / kWave];
  __shared__ int s_wall[256 / kWave];
  __shared__ int s_head_row;
  __shared__ double s_head_val;
  const int tid = threadIdx.x;
  const long long total = static_cast<long long>(nrows) + nnz;
  const long long d0 = static_cast<long long>(blockIdx.x) * TILE;
  const long long d1 = min(d0 + TILE, total);
  const int xb = sc.coord[blockIdx.x];
  const int xe = sc.coord[blockIdx.x + 1];
  const int yb = static_cast<int>(d0 - xb);
  const int ye = static_cast<int>(d1 - xe);
  const int na = max(0, min(xe - xb, TILE));
  const int nb = max(0, min(ye - yb, TILE));
  if (tid == 0) s_head_row = -1;
  // Stage the tile with every load of a thread in flight at once: IPT column
  // indices and values, then the IPT gathers of x, then the row ends.
  // (Plain loads: non-temporal hints measured slower on gfx950.)
  int cidx[IPT];
  float v[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int i = tid + j * 256;
    cidx[j] = i < nb ? col[yb + i] : 0;
    v[j] = i < nb ? val[yb + i] : 0.0f;
  }
  float xv[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) xv[j] = x[min(max(cidx[j], 0), ncols - 1)];
#pragma unroll
  for (int j = 0; j < IPT + 1; ++j) {
    const int i = tid + j * 256;
    if (i <= na) {
      const int r = xb + i;
      s_rowend[i] = r < nrows ? clamp_nnz(row_ptr[r + 1], nnz) : nnz;
    }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int i = tid + j * 256;
    if (i < nb) s_prod[i] = static_cast<double>(v[j]) * static_cast<double>(xv[j]);
  }
  __syncthreads();
  // this thread's segment of the merge path inside the tile
  const int td = min(tid * IPT, na + nb);
  int lo = max(0, td - nb), hi = min(td, na);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s_rowend[mid] <= yb + td - mid - 1)
      lo = mid + 1;
    else
      hi = mid;
  }
  int tx = lo, ty = td - lo;
  const int te = min(td + IPT, na + nb);
  double acc = 0.0;
  bool has_head = false;
  int head_row = 0;
  double head_acc = 0.0;
  for (int d = td; d < te; ++d) {
    if (tx < na && (ty >= nb || s_rowend[tx] <= yb + ty)) {
      if (!has_head) {
        has_head = true;
        head_row = tx;
        head_acc = acc;
      } else {
        s_out[tx] = static_cast<float>(acc);
      }
      acc = 0.0;
      ++tx;
    } else {
      acc += s_prod[ty];
      ++ty;
    }
  }
  // Carries: thread t ends inside row `crow` with partial sum `cval`.  A
  // segmented inclusive scan over threads (rows are non-decreasing, so equal
  // rows are contiguous) gives each thread the sum of the run of same-row
  // carries ending at it: shuffles inside each wave, then one pass over the
  // (at most 3) preceding waves' trailing runs.
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int crow = tx;
  double cval = acc;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double vu = __shfl_up(cval, off, kWave);
    const int ru = __shfl_up(crow, off, kWave);
    if (lane >= off && ru == crow) cval += vu;
  }
  const double prev_v = __shfl_up(cval, 1, kWave);
  const int prev_r = __shfl_up(crow, 1, kWave);
  const int row0 = __shfl(crow, 0, kWave);
  if (lane == kWave - 1) {
    s_wrow[wv] = crow;
    s_wsum[wv] = cval;
    s_wall[wv] = row0 == crow ? 1 : 0;
  }
  __syncthreads();
  // sum of the trailing same-row runs of the waves before this one
  auto from_prev_waves = [&](int row) {
    double c = 0.0;
    for (int w2 = wv - 1; w2 >= 0; --w2) {
      if (s_wrow[w2] != row) break;
      c += s_wsum[w2];
      if (!s_wall[w2]) break;
    }
    return c;
  };
  if (has_head) {
    double cin = (lane > 0 && prev_r == head_row) ? prev_v : 0.0;
    if (lane == 0 || row0 == head_row) cin += from_prev_waves(head_row);
    const double v = head_acc + cin;
    const int grow = xb + head_row;
    if (head_row == 0 && clamp_nnz(row_ptr[xb], nnz) < yb) {
      s_head_row = grow;
      s_head_val = v;
    } else {
      s_out[head_row] = static_cast<float>(v);
    }
  }
  double tail = 0.0;
  if (tid == 255) tail = cval + (row0 == crow ? from_prev_waves(crow) : 0.0);
  __syncthreads();
  // rows [xb, xb + na) end in this tile; the first one is written by the
  // fix-up kernel instead when it started in an earlier tile
  for (int i = (s_head_row >= 0 ? 1 : 0) + tid; i < na; i += 256) y[xb + i] = s_out[i];
  if (tid == 255) {
    sc.head_row[blockIdx.x] = s_head_row;
    sc.head_val[blockIdx.x] = s_head_row >= 0 ? s_head_val : 0.0;
    sc.tail_row[blockIdx.x] = xb + na;
    sc.tail_val[blockIdx.x] = tail;
  }
}

// Rows split across tiles: one wave per tile whose first row started in an
// earlier tile adds the parts of that row held by the preceding tiles, in a
// fixed order.  Row r enters the merge path at diagonal r + row_ptr[r], so
// the first tile whose end reaches that diagonal is the first with a part of
// it (a tile ending exactly there holds an empty part): no search is needed.
__global__ __launch_bounds__(256) void k_spmv_fixup(const int* __restrict__ row_ptr, float* __restrict__ y,
                                                    SpmvScratch sc, int ntiles, int nnz, int tile) {
  const int b = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (b >= ntiles) return;
  const int r = sc.head_row[b];
  if (r < 0 || b == 0) return;
  const long long dr = static_cast<long long>(r) + clamp_nnz(row_ptr[r], nnz);
  const int p0 = static_cast<int>(min(static_cast<long long>(b), max(0LL, (dr + tile - 1) / tile - 1)));
  double acc = 0.0;
  for (int p = p0 + lane; p < b; p += kWave) acc += sc.tail_val[p];
  acc = wave_sum(acc);
  if (lane == 0) y[r] = static_cast<float>(sc.head_val[b] + acc);
}

// Row-window SpMV (the launch variants 0x100 | IPT; 0x200 added: the column
// indices and values are read with non-temporal loads; 0x400: the resident
// grid form below).  Tile b covers the
// nonzeros [b*W, min((b+1)*W, nnz)), W = 256 * IPT, and owns the rows that
// start in that window (own[b] <= r < own[b+1]; the last tile also owns the
// rows that start at nnz).  The tile's products are formed coalesced (IPT
// column indices and values per thread, their gathers of x, fp64 products in
// LDS); then each owned row is summed from LDS, by one thread when its part
// in the tile has at most kShortRow nonzeros and by a whole wave (strided
// lanes, butterfly) otherwise.  The only owned row that can run past the
// tile is the last one: its in-tile sum is the tile's tail part.  Nonzeros at
// the start of the tile that belong to a row started in an earlier tile are
// summed by wave 0 into the tile's head part; the fix-up adds the parts of
// such a row in tile order, in the tile where the row ends.  Every sum is
// taken in a fixed order, so results do not depend on timing.
constexpr int kShortRow = 32;

struct SpmvWindowScratch {
  double* head_val;  // per tile: sum of the nonzeros before its first owned row
  double* tail_val;  // per tile: in-tile sum of its last owned row when that row runs past the tile
  int* head_row;     // per tile: the row its head part ends (fix-up writes it), else -1
};

// Smallest r in [0, nrows] with row_ptr[r] >= target (r = nrows when no row
// starts at or after target), by one wave: 64 probes per round shrink the
// interval 65-fold.
__device__ int wave_lower_bound(const int* __restrict__ row_ptr, int nrows, int nnz, long long target) {
  const int lane = threadIdx.x & (kWave - 1);
  int lo = 0, hi = nrows;  // the answer lies in [lo, hi]
  while (hi - lo > kWave) {
    const long long span = hi - lo;
    const int xq = lo + static_cast<int>(((lane + 1) * span) / (kWave + 1));  // lo < xq < hi
    const bool below = clamp_nnz(row_ptr[xq], nnz) < target;
    const int c = __popcll(__ballot(below));  // probes 0 .. c-1 lie below the target
    const int lo0 = lo;
    if (c > 0) lo = lo0 + static_cast<int>((c * span) / (kWave + 1)) + 1;
    if (c < kWave) hi = lo0 + static_cast<int>(((c + 1) * span) / (kWave + 1));
  }
  const int xq = lo + lane;
  const bool below = xq < hi && clamp_nnz(row_ptr[xq], nnz) < target;
  return lo + __popcll(__ballot(below));
}

// own[b] for b = 0 .. ntiles (own[ntiles] = nrows), one wave per boundary.
__global__ __launch_bounds__(256) void k_spmv_window_partition(const int* __restrict__ row_ptr, int nrows,
                                                               int nnz, int window, int ntiles,
                                                               int* __restrict__ own) {
  const int b = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (b > ntiles) return;
  const int r = b == ntiles ? nrows : wave_lower_bound(row_ptr, nrows, nnz, static_cast<long long>(b) * window);
  if ((threadIdx.x & (kWave - 1)) == 0) own[b] = r;
}

// The row phase of a row-window tile whose products are in s_prod: the
// tile's head part (wave 0), then its owned rows r0 .. r1 - 1.  The values
// it needs first come in with the matrix: pre_s, pre_e are the bounds of row
// r0 + tid and head_end the start of row r0 (nnz if r0 = nrows), so the
// usual tile makes no global load here (rows past the first 256 load their
// bounds).  Long rows are handed to the waves through LDS with their bounds
// (s_long: 4 ints each).  Every thread takes part (the barriers inside are
// reached by all).
__device__ __forceinline__ void spmv_window_rows(const int* __restrict__ row_ptr, float* __restrict__ y, int nrows,
                                                 int nnz, int b, int k0, int k1, int r0, int r1, int pre_s,
                                                 int pre_e, int head_end, const double* s_prod, int* s_long,
                                                 int* s_nlong, SpmvWindowScratch sc) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  // local [start, end) of a row's nonzeros [s0, e) inside the tile
  auto clip = [&](int s0, int e, int* ls, int* le) {
    *ls = min(max(s0, k0), k1) - k0;
    *le = max(min(max(e, k0), k1) - k0, *ls);
  };
  auto local_range = [&](int r, int* ls, int* le, int* e) {
    *e = clamp_nnz(row_ptr[r + 1], nnz);
    clip(clamp_nnz(row_ptr[r], nnz), *e, ls, le);
  };
  if (wv == 0) {
    const int hend = min(max(head_end, k0), k1);
    double h = 0.0;
    for (int i = lane; i < hend - k0; i += kWave) h += s_prod[i];
    h = wave_sum(h);
    if (lane == 0) {
      sc.head_val[b] = h;
      // the head part ends its row here unless the row runs on past the tile
      const bool has_head = b > 0 && r0 > 0 && hend > k0;
      const bool ends_here = head_end <= k1;
      sc.head_row[b] = has_head && ends_here ? r0 - 1 : -1;
    }
  }
  for (int c = r0; c < r1; c += 256) {
    const int r = c + tid;
    if (r < r1) {
      int ls, le, e;
      if (c == r0) {
        e = pre_e;
        clip(pre_s, pre_e, &ls, &le);
      } else {
        local_range(r, &ls, &le, &e);
      }
      if (le - ls <= kShortRow) {
        double acc = 0.0;
        for (int i = ls; i < le; ++i) acc += s_prod[i];
        if (e <= k1)
          y[r] = static_cast<float>(acc);
        else
          sc.tail_val[b] = acc;
      } else {
        int* slot = s_long + 4 * atomicAdd(s_nlong, 1);
        slot[0] = r;
        slot[1] = ls;
        slot[2] = le;
        slot[3] = e;
      }
    }
    __syncthreads();
    const int nl = *s_nlong;
    for (int q = wv; q < nl; q += 256 / kWave) {
      const int r2 = s_long[4 * q], ls = s_long[4 * q + 1], le = s_long[4 * q + 2], e = s_long[4 * q + 3];
      double acc = 0.0;
      for (int i = ls + lane; i < le; i += kWave) acc += s_prod[i];
      acc = wave_sum(acc);
      if (lane == 0) {
        if (e <= k1)
          y[r2] = static_cast<float>(acc);
        else
          sc.tail_val[b] = acc;
      }
    }
    __syncthreads();
    if (tid == 0) *s_nlong = 0;
    __syncthreads();
  }
}

template <int IPT, bool kStream>
__global__ __launch_bounds__(256) void k_spmv_window(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                     const float* __restrict__ val, const float* __restrict__ x,
                                                     float* __restrict__ y, int nrows, int ncols, int nnz,
                                                     const int* __restrict__ own, SpmvWindowScratch sc) {
  constexpr int W = 256 * IPT;
  __shared__ double s_prod[W];
  __shared__ int s_long[4 * 256];
  __shared__ int s_nlong;
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int k0 = static_cast<int>(min(static_cast<long long>(b) * W, static_cast<long long>(nnz)));
  const int k1 = static_cast<int>(min(static_cast<long long>(k0) + W, static_cast<long long>(nnz)));
  const int cnt = k1 - k0;
  // the first 256 owned rows' bounds are loaded while the matrix is
  const int r0 = own[b], r1 = own[b + 1];
  int pre_s = 0, pre_e = 0;
  if (r0 + tid < r1) {
    pre_s = clamp_nnz(row_ptr[r0 + tid], nnz);
    pre_e = clamp_nnz(row_ptr[r0 + tid + 1], nnz);
  }
  const int head_end = r0 < nrows ? clamp_nnz(row_ptr[r0], nnz) : nnz;
  int cidx[IPT];
  float v[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int i = tid + j * 256;
    if (kStream) {  // read once: hint the caches to keep x's lines rather than these
      cidx[j] = i < cnt ? __builtin_nontemporal_load(col + k0 + i) : 0;
      v[j] = i < cnt ? __builtin_nontemporal_load(val + k0 + i) : 0.0f;
    } else {
      cidx[j] = i < cnt ? col[k0 + i] : 0;
      v[j] = i < cnt ? val[k0 + i] : 0.0f;
    }
  }
  float xv[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) xv[j] = x[min(max(cidx[j], 0), ncols - 1)];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int i = tid + j * 256;
    if (i < cnt) s_prod[i] = static_cast<double>(v[j]) * static_cast<double>(xv[j]);
  }
  if (tid == 0) s_nlong = 0;
  __syncthreads();
  spmv_window_rows(row_ptr, y, nrows, nnz, b, k0, k1, r0, r1, pre_s, pre_e, head_end, s_prod, s_long, &s_nlong, sc);
}

// The same tiles, a resident grid looping over them: while one tile's rows
// are summed from LDS, the matrix, row bounds and owned-row range of the
// workgroup's next tile are already being loaded (variant bit 0x400).
template <int IPT>
__global__ __launch_bounds__(256) void k_spmv_window_pf(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                        const float* __restrict__ val, const float* __restrict__ x,
                                                        float* __restrict__ y, int nrows, int ncols, int nnz,
                                                        const int* __restrict__ own, int ntiles,
                                                        SpmvWindowScratch sc) {
  constexpr int W = 256 * IPT;
  __shared__ double s_prod[W];
  __shared__ int s_long[4 * 256];
  __shared__ int s_nlong;
  const int tid = threadIdx.x;
  auto window = [&](int t, int* k0, int* k1) {
    *k0 = static_cast<int>(min(static_cast<long long>(t) * W, static_cast<long long>(nnz)));
    *k1 = static_cast<int>(min(static_cast<long long>(*k0) + W, static_cast<long long>(nnz)));
  };
  // tile t's matrix slice, owned rows and the bounds the row phase starts with
  auto load = [&](int t, int (&ci)[IPT], float (&vv)[IPT], int* r0, int* r1, int* ps, int* pe, int* he) {
    int k0, k1;
    window(t, &k0, &k1);
    const int cnt = k1 - k0;
    *r0 = own[t];
    *r1 = own[t + 1];
    *ps = 0;
    *pe = 0;
    if (*r0 + tid < *r1) {
      *ps = clamp_nnz(row_ptr[*r0 + tid], nnz);
      *pe = clamp_nnz(row_ptr[*r0 + tid + 1], nnz);
    }
    *he = *r0 < nrows ? clamp_nnz(row_ptr[*r0], nnz) : nnz;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = tid + j * 256;
      ci[j] = i < cnt ? col[k0 + i] : 0;
      vv[j] = i < cnt ? val[k0 + i] : 0.0f;
    }
  };
  int cidx[IPT];
  float v[IPT];
  int r0 = 0, r1 = 0, ps = 0, pe = 0, he = 0;
  int b = blockIdx.x;
  if (b < ntiles) load(b, cidx, v, &r0, &r1, &ps, &pe, &he);
  if (tid == 0) s_nlong = 0;
  for (; b < ntiles; b += gridDim.x) {
    int k0, k1;
    window(b, &k0, &k1);
    const int cnt = k1 - k0;
    float xv[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) xv[j] = x[min(max(cidx[j], 0), ncols - 1)];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int i = tid + j * 256;
      if (i < cnt) s_prod[i] = static_cast<double>(v[j]) * static_cast<double>(xv[j]);
    }
    const int nb = b + static_cast<int>(gridDim.x);
    int ncidx[IPT];
    float nv[IPT];
    int nr0 = 0, nr1 = 0, nps = 0, npe = 0, nhe = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      ncidx[j] = 0;
      nv[j] = 0.0f;
    }
    if (nb < ntiles) load(nb, ncidx, nv, &nr0, &nr1, &nps, &npe, &nhe);
    __syncthreads();
    spmv_window_rows(row_ptr, y, nrows, nnz, b, k0, k1, r0, r1, ps, pe, he, s_prod, s_long, &s_nlong, sc);
    __syncthreads();  // s_prod is rewritten by the next tile
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      cidx[j] = ncidx[j];
      v[j] = nv[j];
    }
    r0 = nr0;
    r1 = nr1;
    ps = nps;
    pe = npe;
    he = nhe;
  }
}

// Rows that run across tiles: for each tile b whose head part ends a row,
// y[row] = (the row's tail part in the tile that owns it) + (the head parts
// of tiles owner + 1 .. b).  One thread per tile: a row spanning at most
// kFixupSerial tiles (nearly all: a tile holds 1024 or 2048 nonzeros) is
// summed by its thread in tile order; longer ones go to the whole wave, one
// at a time, with a fixed lane-strided order and butterfly.  Few, short
// workgroups, so that the kernel is not held back when another kernel fills
// the GPU beside it.
constexpr int kFixupSerial = 8;

__global__ __launch_bounds__(256) void k_spmv_window_fixup(const int* __restrict__ row_ptr, float* __restrict__ y,
                                                           SpmvWindowScratch sc, int ntiles, int nnz, int window) {
  const int b = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  const int lane = static_cast<int>(threadIdx.x & (kWave - 1));
  int r = -1, owner = 0;
  if (b < ntiles) {
    r = sc.head_row[b];
    if (r >= 0) owner = min(clamp_nnz(row_ptr[r], nnz) / window, ntiles - 1);
  }
  const bool alone = r >= 0 && b - owner <= kFixupSerial;
  if (alone) {
    double acc = 0.0;
    for (int k = owner + 1; k <= b; ++k) acc += sc.head_val[k];
    y[r] = static_cast<float>(sc.tail_val[owner] + acc);
  }
  uint64_t rest = __ballot(r >= 0 && !alone);  // every lane of the wave takes part from here on
  while (rest) {
    const int l = __ffsll(static_cast<unsigned long long>(rest)) - 1;
    rest &= rest - 1;
    const int bl = __shfl(b, l, kWave), rl = __shfl(r, l, kWave), ol = __shfl(owner, l, kWave);
    double acc = 0.0;
    for (int k = ol + 1 + lane; k <= bl; k += kWave) acc += sc.head_val[k];
    acc = wave_sum(acc);
    if (lane == 0) y[rl] = static_cast<float>(sc.tail_val[ol] + acc);
  }
}

// CSR SpMV for matrices with short rows: L lanes per row stride over the row
// (the matrix read once, coalesced within the row), fp64 partial sums
// combined by an xor butterfly inside each group of L lanes.  No search and
// no LDS; a row of length m costs m / L iterations, so it is meant for
// bounded row lengths (e.g. a fixed out-degree).
template <int L>
__global__ __launch_bounds__(256) void k_spmv_rows(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                   const float* __restrict__ val, const float* __restrict__ x,
                                                   float* __restrict__ y, int nrows, int ncols, int nnz) {
  const int lane = threadIdx.x & (L - 1);
  const long long stride = static_cast<long long>(gridDim.x) * (256 / L);
  for (long long r = (static_cast<long long>(blockIdx.x) * 256 + threadIdx.x) / L; r < nrows; r += stride) {
    const int b = clamp_nnz(row_ptr[r], nnz), e = clamp_nnz(row_ptr[r + 1], nnz);
    double acc = 0.0;
    for (int k = b + lane; k < e; k += L)
      acc += static_cast<double>(val[k]) * static_cast<double>(x[min(max(col[k], 0), ncols - 1)]);
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[r] = static_cast<float>(acc);
  }
}

// s = sum v_i^2 (fp64).
template <bool kSinglePass>
__global__ __launch_bounds__(1024) void k_sumsq(const float* __restrict__ v, double* __restrict__ s,
                                                uint64_t n, int vec, uint32_t* counter,
                                                uint64_t* partials) {
  __shared__ double sh[17];
  __shared__ int flag;
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  double acc = 0.0;
  uint64_t start = 0;
  if (vec) {
    const float4* v4 = reinterpret_cast<const float4*>(v);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 a = v4[i];
      const double ax = a.x, ay = a.y, az = a.z, aw = a.w;
      acc += ax * ax;
      acc += ay * ay;
      acc += az * az;
      acc += aw * aw;
    }
    start = n4 << 2;
  }
  for (uint64_t i = start + gid; i < n; i += stride) {
    const double a = v[i];
    acc += a * a;
  }
  const double bsum = block_sum(acc, sh);
  publish_partial(partials, d2u(bsum));
  if (kSinglePass && arrive_last(counter, &flag)) {
    double t = 0.0;
    for (uint32_t i = threadIdx.x; i < gridDim.x; i += blockDim.x) t += u2d(read_partial(partials, i));
    const double tot = block_sum(t, sh);
    if (threadIdx.x == 0) s[0] = tot;
    reset_counter(counter);
  }
}

// v_i = fl32(t_i / sqrt(s)) in fp64.
__global__ __launch_bounds__(1024) void k_scale_l2(const float* __restrict__ t,
                                                   const double* __restrict__ s,
                                                   float* __restrict__ v, uint64_t n, int vec) {
  const double r = sqrt(s[0]);
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t start = 0;
  if (vec) {
    const float4* t4 = reinterpret_cast<const float4*>(t);
    float4* v4 = reinterpret_cast<float4*>(v);
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride) {
      const float4 a = t4[i];
      v4[i] = make_float4(static_cast<float>(a.x / r), static_cast<float>(a.y / r),
                          static_cast<float>(a.z / r), static_cast<float>(a.w / r));
    }
    start = n4 << 2;
  }
  for (uint64_t i = start + gid; i < n; i += stride) v[i] = static_cast<float>(t[i] / r);
}

// ---------------------------------------------------------------------------
// ML ensemble (Sec. V-B): categorical naive Bayes and a ridge classifier
// score the same rows of X (n rows x F features of fp32 category codes);
// each row of C scores becomes probabilities by a softmax; the two
// probability rows are averaged and reduced to the index of the largest
// average.
//
// X is stored feature-major (feature f of row r at X[f*n + r]) and a thread
// owns one row, so the 64 lanes of a wave read 256 contiguous bytes per
// feature and the per-feature model data are the same for the whole wave.
// kMlUnroll loads are issued before they are used.
// ---------------------------------------------------------------------------
constexpr int kMlMaxClasses = 16;
constexpr int kMlUnroll = 8;               // features loaded ahead per lane
constexpr uint32_t kNbTable = 32768;       // C*F*V fp32 entries of the naive Bayes table (128 KB)
constexpr uint32_t kRidgeLdsBytes = 65536; // F*(C+1) fp64: weights / scale, then means

// P = softmax(s) rounded to fp32: the largest score is subtracted before exp.
template <int C>
__device__ __forceinline__ void softmax_store(double (&s)[C], float* __restrict__ out) {
  double m = s[0];
#pragma unroll
  for (int c = 1; c < C; ++c) m = fmax(m, s[c]);
  double tot = 0.0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    s[c] = exp(s[c] - m);
    tot += s[c];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) out[c] = static_cast<float>(s[c] / tot);
}

// acc[c] += log theta[c][f][code(x)] for one feature; t points at feature f's
// block of the LDS table ([v][c], C values per code).  Codes are truncated and
// clamped to [0, V-1] so that no input can address outside the table.
template <int C>
__device__ __forceinline__ void nb_add(double (&acc)[C], const float* __restrict__ t, float vmax, float x) {
  const int v = static_cast<int>(fminf(fmaxf(x, 0.0f), vmax));
  const float* e = t + v * C;
  if constexpr (C % 2 == 0) {
#pragma unroll
    for (int c = 0; c < C; c += 2) {
      const float2 p = *reinterpret_cast<const float2*>(e + c);
      acc[c] += static_cast<double>(p.x);
      acc[c + 1] += static_cast<double>(p.y);
    }
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += static_cast<double>(e[c]);
  }
}

template <int C>
__global__ __launch_bounds__(1024) void k_nb_proba(const float* __restrict__ X, const float* __restrict__ lt,
                                                   const float* __restrict__ lp, float* __restrict__ P,
                                                   uint64_t n, uint32_t F, uint32_t V) {
  __shared__ __align__(16) float s_tab[kNbTable];  // [f][v][c]
  const uint32_t fv_n = F * V;
  for (uint32_t i = threadIdx.x; i < C * fv_n; i += blockDim.x) {
    const uint32_t c = i / fv_n;
    s_tab[(i - c * fv_n) * C + c] = lt[i];  // lt is [c][f][v]
  }
  __syncthreads();
  double prior[C];
#pragma unroll
  for (int c = 0; c < C; ++c) prior[c] = static_cast<double>(lp[c]);
  const float vmax = static_cast<float>(V - 1);
  const uint32_t tstride = V * C;  // table floats per feature
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < n; r += stride) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = prior[c];
    const float* col = X + r;
    uint32_t f = 0;
    for (; f + kMlUnroll <= F; f += kMlUnroll) {
      float x[kMlUnroll];
#pragma unroll
      for (int u = 0; u < kMlUnroll; ++u) x[u] = col[static_cast<uint64_t>(f + u) * n];
#pragma unroll
      for (int u = 0; u < kMlUnroll; ++u) nb_add<C>(acc, s_tab + (f + u) * tstride, vmax, x[u]);
    }
    for (; f < F; ++f) nb_add<C>(acc, s_tab + f * tstride, vmax, col[static_cast<uint64_t>(f) * n]);
    softmax_store<C>(acc, P + r * C);
  }
}

// acc[c] += (x - mean_f) * (W[c][f] / scale_f) for one feature (w = that
// feature's C weights in LDS, the same address for every lane).
template <int C>
__device__ __forceinline__ void ridge_add(double (&acc)[C], const double* __restrict__ w, double d) {
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = fma(d, w[c], acc[c]);
}

template <int C>
__global__ __launch_bounds__(512) void k_ridge_proba(const float* __restrict__ X, const float* __restrict__ mean,
                                                     const float* __restrict__ scale, const float* __restrict__ W,
                                                     const float* __restrict__ b, float* __restrict__ P,
                                                     uint64_t n, uint32_t F) {
  extern __shared__ __align__(16) double s_w[];  // [f][c] weights / scale, then F means
  double* s_mu = s_w + F * C;
  for (uint32_t i = threadIdx.x; i < C * F; i += blockDim.x) {
    const uint32_t c = i / F, f = i - c * F;  // W is [c][f]
    s_w[f * C + c] = static_cast<double>(W[i]) / static_cast<double>(scale[f]);
  }
  for (uint32_t f = threadIdx.x; f < F; f += blockDim.x) s_mu[f] = static_cast<double>(mean[f]);
  __syncthreads();
  double bias[C];
#pragma unroll
  for (int c = 0; c < C; ++c) bias[c] = static_cast<double>(b[c]);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < n; r += stride) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = bias[c];
    const float* col = X + r;
    // the next kMlUnroll features are loaded while the current ones are used
    uint32_t f = 0;
    float x[kMlUnroll];
    if (F >= static_cast<uint32_t>(kMlUnroll)) {
#pragma unroll
      for (int u = 0; u < kMlUnroll; ++u) x[u] = col[static_cast<uint64_t>(u) * n];
    }
#pragma unroll 1
    for (; f + kMlUnroll <= F; f += kMlUnroll) {
      float xn[kMlUnroll];
      const bool more = f + 2 * kMlUnroll <= F;
      if (more) {
#pragma unroll
        for (int u = 0; u < kMlUnroll; ++u) xn[u] = col[static_cast<uint64_t>(f + kMlUnroll + u) * n];
      }
#pragma unroll
      for (int u = 0; u < kMlUnroll; ++u)
        ridge_add<C>(acc, s_w + (f + u) * C, static_cast<double>(x[u]) - s_mu[f + u]);
      if (more) {
#pragma unroll
        for (int u = 0; u < kMlUnroll; ++u) x[u] = xn[u];
      }
    }
    for (; f < F; ++f) ridge_add<C>(acc, s_w + f * C, static_cast<double>(col[static_cast<uint64_t>(f) * n]) - s_mu[f]);
    softmax_store<C>(acc, P + r * C);
  }
}

// Four consecutive rows per thread with 16-byte loads (n a multiple of 4,
// X 16-byte aligned): a wave reads 1 KB contiguous per feature, twice the
// bytes in flight of two single rows, and the weights read from LDS serve
// four rows.
template <int C>
__global__ __launch_bounds__(256) void k_ridge_proba4(const float* __restrict__ X, const float* __restrict__ mean,
                                                      const float* __restrict__ scale, const float* __restrict__ W,
                                                      const float* __restrict__ b, float* __restrict__ P,
                                                      uint64_t n, uint32_t F) {
  extern __shared__ __align__(16) double s_w[];  // [f][c] weights / scale, then F means
  double* s_mu = s_w + F * C;
  for (uint32_t i = threadIdx.x; i < C * F; i += blockDim.x) {
    const uint32_t c = i / F, f = i - c * F;  // W is [c][f]
    s_w[f * C + c] = static_cast<double>(W[i]) / static_cast<double>(scale[f]);
  }
  for (uint32_t f = threadIdx.x; f < F; f += blockDim.x) s_mu[f] = static_cast<double>(mean[f]);
  __syncthreads();
  double bias[C];
#pragma unroll
  for (int c = 0; c < C; ++c) bias[c] = static_cast<double>(b[c]);
  const uint64_t groups = n / 4;  // float4 columns per feature
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t g = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; g < groups; g += stride) {
    double acc[4][C];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[j][c] = bias[c];
    const float4* col = X4 + g;
    // the next kU4 features are loaded while the current ones are used
    constexpr int kU4 = kMlUnroll / 2;
    uint32_t f = 0;
    // loads ahead clamped to the last feature, so the body has no branch
    float4 x[kU4];
#pragma unroll
    for (int u = 0; u < kU4; ++u) x[u] = col[static_cast<uint64_t>(min(static_cast<uint32_t>(u), F - 1)) * groups];
#pragma unroll 1
    for (; f + kU4 <= F; f += kU4) {
      float4 xn[kU4];
#pragma unroll
      for (int u = 0; u < kU4; ++u) xn[u] = col[static_cast<uint64_t>(min(f + kU4 + u, F - 1)) * groups];
#pragma unroll
      for (int u = 0; u < kU4; ++u) {
        const double mu = s_mu[f + u];
        const double* w = s_w + (f + u) * C;
        ridge_add<C>(acc[0], w, static_cast<double>(x[u].x) - mu);
        ridge_add<C>(acc[1], w, static_cast<double>(x[u].y) - mu);
        ridge_add<C>(acc[2], w, static_cast<double>(x[u].z) - mu);
        ridge_add<C>(acc[3], w, static_cast<double>(x[u].w) - mu);
      }
#pragma unroll
      for (int u = 0; u < kU4; ++u) x[u] = xn[u];
    }
    for (; f < F; ++f) {
      const float4 x = col[static_cast<uint64_t>(f) * groups];
      const double mu = s_mu[f];
      const double* w = s_w + f * C;
      ridge_add<C>(acc[0], w, static_cast<double>(x.x) - mu);
      ridge_add<C>(acc[1], w, static_cast<double>(x.y) - mu);
      ridge_add<C>(acc[2], w, static_cast<double>(x.z) - mu);
      ridge_add<C>(acc[3], w, static_cast<double>(x.w) - mu);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) softmax_store<C>(acc[j], P + (4 * g + j) * C);
  }
}

// Two consecutive rows per thread with 8-byte loads (n even, X 8-byte
// aligned) and eight features in flight: the four-row kernel needs about 250
// registers (two waves per SIMD); two rows' accumulators and the loads in
// flight fit in 128 (four waves).  Same sums in the same order as the
// one-row kernel.
template <int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ridge_proba2(
    const float* __restrict__ X, const float* __restrict__ mean, const float* __restrict__ scale,
    const float* __restrict__ W, const float* __restrict__ b, float* __restrict__ P, uint64_t n, uint32_t F) {
  extern __shared__ __align__(16) double s_w[];  // [f][c] weights / scale, then F means
  double* s_mu = s_w + F * C;
  for (uint32_t i = threadIdx.x; i < C * F; i += blockDim.x) {
    const uint32_t c = i / F, f = i - c * F;  // W is [c][f]
    s_w[f * C + c] = static_cast<double>(W[i]) / static_cast<double>(scale[f]);
  }
  for (uint32_t f = threadIdx.x; f < F; f += blockDim.x) s_mu[f] = static_cast<double>(mean[f]);
  __syncthreads();
  const uint64_t pairs = n / 2;  // float2 columns per feature
  const float2* X2 = reinterpret_cast<const float2*>(X);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  constexpr int kU = 8;
  for (uint64_t g = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; g < pairs; g += stride) {
    double acc[2][C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[0][c] = acc[1][c] = static_cast<double>(b[c]);
    const float2* col = X2 + g;
    uint32_t f = 0;
    // the loads ahead are clamped to the last feature instead of skipped, so
    // the loop body has no branch (a branch there split it, and the compiler
    // then hoisted every feature's weight reads and spilled)
    float2 x[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = col[static_cast<uint64_t>(min(static_cast<uint32_t>(u), F - 1)) * pairs];
#pragma unroll 1
    for (; f + kU <= F; f += kU) {
      float2 xn[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) xn[u] = col[static_cast<uint64_t>(min(f + kU + u, F - 1)) * pairs];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const double mu = s_mu[f + u];
        const double* w = s_w + (f + u) * C;
        ridge_add<C>(acc[0], w, static_cast<double>(x[u].x) - mu);
        ridge_add<C>(acc[1], w, static_cast<double>(x[u].y) - mu);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) x[u] = xn[u];
    }
    for (; f < F; ++f) {
      const float2 xv = col[static_cast<uint64_t>(f) * pairs];
      const double mu = s_mu[f];
      const double* w = s_w + f * C;
      ridge_add<C>(acc[0], w, static_cast<double>(xv.x) - mu);
      ridge_add<C>(acc[1], w, static_cast<double>(xv.y) - mu);
    }
    softmax_store<C>(acc[0], P + (2 * g) * C);
    softmax_store<C>(acc[1], P + (2 * g + 1) * C);
  }
}

// avg = (a + b) / 2, exact in fp64, stored rounded to fp32; label = first
// index of the largest fp64 average (lowest class on ties).
template <int C>
__global__ __launch_bounds__(1024) void k_ensemble(const float* __restrict__ pa, const float* __restrict__ pb,
                                                   float* __restrict__ avg, int* __restrict__ label, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < n; r += stride) {
    const float* a = pa + r * C;
    const float* b = pb + r * C;
    float* o = avg + r * C;
    double best = -INFINITY;
    int arg = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double m = (static_cast<double>(a[c]) + static_cast<double>(b[c])) * 0.5;
      o[c] = static_cast<float>(m);
      if (m > best) {
        best = m;
        arg = c;
      }
    }
    label[r] = arg;
  }
}

// ---------------------------------------------------------------------------
// DL (Sec. V-B): a Siamese convolutional network.  Tensors are channel-major
// (C, H, W) fp32; arithmetic in fp64, one rounding to fp32 per output.
//
// 3x3 convolution (zero padding) + bias + ReLU + 2x2 max pooling in one
// kernel: a 256-thread workgroup owns a 16 x 16 tile of pooled outputs (a
// 32 x 32 tile of convolution outputs) for OC output channels.  Per input
// channel the 34 x 34 input tile and the OC x 9 weights (as fp64) are staged
// in LDS once and serve all OC channels; each thread keeps its 4 convolution
// outputs per channel in fp64 registers, and ReLU then max equals max then
// ReLU (ReLU is monotone).
// ---------------------------------------------------------------------------
constexpr int kConvTile = 16;  // pooled outputs per tile side

template <int OC>
__global__ __launch_bounds__(256) void k_conv3x3_relu_pool(const float* __restrict__ x, const float* __restrict__ w,
                                                           const float* __restrict__ bias, float* __restrict__ y,
                                                           uint32_t cin, uint32_t h, uint32_t wd,
                                                           uint32_t tiles_x) {
  constexpr int kIn = 2 * kConvTile + 2;  // 34 input rows / columns per tile
  __shared__ float s_in[kIn][kIn + 1];
  __shared__ double s_w[OC * 9];          // this input channel's weights of the OC output channels
  const uint32_t ph = h / 2, pw = wd / 2;
  const uint32_t ty0 = (blockIdx.x / tiles_x) * kConvTile, tx0 = (blockIdx.x % tiles_x) * kConvTile;
  const uint32_t o0 = blockIdx.y * OC;
  const uint32_t tx = threadIdx.x % kConvTile, ty = threadIdx.x / kConvTile;
  const int gy0 = 2 * static_cast<int>(ty0) - 1, gx0 = 2 * static_cast<int>(tx0) - 1;
  double acc[OC][4];
#pragma unroll
  for (int k = 0; k < OC; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[k][q] = static_cast<double>(bias[o0 + k]);
  for (uint32_t c = 0; c < cin; ++c) {
    const float* xc = x + static_cast<uint64_t>(c) * h * wd;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kIn * kIn; i += blockDim.x) {
      const int r = static_cast<int>(i / kIn), q = static_cast<int>(i % kIn);
      const int gy = gy0 + r, gx = gx0 + q;
      s_in[r][q] = (gy >= 0 && gy < static_cast<int>(h) && gx >= 0 && gx < static_cast<int>(wd))
                       ? xc[static_cast<uint64_t>(gy) * wd + gx]
                       : 0.0f;
    }
    for (uint32_t i = threadIdx.x; i < OC * 9; i += blockDim.x)
      s_w[i] = static_cast<double>(w[(static_cast<uint64_t>(o0 + i / 9) * cin + c) * 9 + i % 9]);
    __syncthreads();
    double p[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int d = 0; d < 4; ++d) p[a][d] = static_cast<double>(s_in[2 * ty + a][2 * tx + d]);
#pragma unroll
    for (int k = 0; k < OC; ++k) {
      double wv[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) wv[t] = s_w[k * 9 + t];
#pragma unroll
      for (int qy = 0; qy < 2; ++qy)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) {
          double sacc = acc[k][qy * 2 + qx];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) sacc = fma(wv[dy * 3 + dx], p[qy + dy][qx + dx], sacc);
          acc[k][qy * 2 + qx] = sacc;
        }
    }
  }
  const uint32_t py = ty0 + ty, px = tx0 + tx;
  if (py < ph && px < pw) {
#pragma unroll
    for (int k = 0; k < OC; ++k) {
      const double m = fmax(fmax(acc[k][0], acc[k][1]), fmax(acc[k][2], acc[k][3]));
      y[(static_cast<uint64_t>(o0 + k) * ph + py) * pw + px] = static_cast<float>(fmax(m, 0.0));
    }
  }
}

// The same convolution with the input channels pipelined: the next
// channel's input tile and weights are fetched into registers while the
// current channel is computed from one half of a double-buffered LDS tile,
// then stored into the other half, so each channel costs one barrier and the
// global-load latency hides behind the FMAs.  The tile is kept flat (row
// stride 34) so that thread t always stages elements t + 256 j; their image
// offsets are computed once (out-of-image elements read offset 0 and store
// zero).  Results equal the unpipelined kernel's bit for bit (same FMA order).
//
// SW (scalar weights): the weights come from an fp64 copy laid out
// [input channel][output channel][9] and are read with uniform (scalar)
// loads straight into the FMAs' scalar operand, instead of being broadcast
// from LDS: a 16-byte broadcast read still returns 1 KB per wave, and 72 of
// them per channel nearly saturate the CU's LDS bandwidth.  (Measured slower
// than the LDS form on every shape tried: the scalar loads' latency shows.)
template <int OC, bool SW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_conv3x3_relu_pool_pipe(
    const float* __restrict__ x, const float* __restrict__ w, const double* __restrict__ w64,
    const float* __restrict__ bias, float* __restrict__ y, uint32_t cin, uint32_t cout, uint32_t h, uint32_t wd,
    uint32_t tiles_x) {
  constexpr int kIn = 2 * kConvTile + 2;        // 34 input rows / columns per tile
  constexpr int kEl = kIn * kIn;                // 1156 tile elements
  constexpr int kSlots = (kEl + 255) / 256;     // 5 staged elements per thread
  // every thread stores all its slots and one weight (threads past the
  // 72 weights store into a spare slot), so the stores need no branch
  constexpr int kW = (OC * 9 + 2) & ~1;         // weights + spare slot, even for 16-byte reads
  __shared__ float s_in[2][kSlots * 256];
  __shared__ __align__(16) double s_w[2][SW ? 2 : kW];
  const uint32_t ph = h / 2, pw = wd / 2;
  const uint32_t ty0 = (blockIdx.x / tiles_x) * kConvTile, tx0 = (blockIdx.x % tiles_x) * kConvTile;
  const uint32_t o0 = blockIdx.y * OC;
  const uint32_t tid = threadIdx.x;
  const uint32_t tx = tid % kConvTile, ty = tid / kConvTile;
  const int gy0 = 2 * static_cast<int>(ty0) - 1, gx0 = 2 * static_cast<int>(tx0) - 1;
  uint32_t off[kSlots];
  uint32_t valid = 0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    const int i = static_cast<int>(tid) + 256 * j;
    const int gy = gy0 + i / kIn, gx = gx0 + i % kIn;
    const bool in = i < kEl && gy >= 0 && gy < static_cast<int>(h) && gx >= 0 && gx < static_cast<int>(wd);
    off[j] = in ? static_cast<uint32_t>(gy) * wd + static_cast<uint32_t>(gx) : 0u;
    valid |= in ? (1u << j) : 0u;
  }
  const bool wl = tid < OC * 9;  // this thread stages one weight per channel
  const uint64_t w0 = wl ? static_cast<uint64_t>(o0 + tid / 9) * cin * 9 + tid % 9 : 0;
  const uint64_t plane = static_cast<uint64_t>(h) * wd;
  float v[kSlots];
  float wr = 0.0f;
  auto fetch = [&](uint32_t c) {
    const float* xc = x + c * plane;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) v[j] = xc[off[j]];
    if constexpr (!SW) wr = w[w0 + 9ull * c];
  };
  auto put = [&](int b) {
#pragma unroll
    for (int j = 0; j < kSlots; ++j) s_in[b][tid + 256 * j] = (valid >> j) & 1u ? v[j] : 0.0f;
    if constexpr (!SW) s_w[b][wl ? tid : kW - 1] = static_cast<double>(wr);
  };
  double acc[OC][4];
#pragma unroll
  for (int k = 0; k < OC; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[k][q] = static_cast<double>(bias[o0 + k]);
  auto compute = [&](int b, uint32_t c) {
    double p[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int d = 0; d < 4; ++d) p[a][d] = static_cast<double>(s_in[b][(2 * ty + a) * kIn + 2 * tx + d]);
#pragma unroll
    for (int k = 0; k < OC; ++k) {
      double wv[9];
#pragma unroll
      for (int t = 0; t < 9; ++t)
        wv[t] = SW ? w64[(static_cast<uint64_t>(c) * cout + o0 + k) * 9 + t] : s_w[b][k * 9 + t];
#pragma unroll
      for (int qy = 0; qy < 2; ++qy)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) {
          double sacc = acc[k][qy * 2 + qx];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) sacc = fma(wv[dy * 3 + dx], p[qy + dy][qx + dx], sacc);
          acc[k][qy * 2 + qx] = sacc;
        }
    }
  };
  // channel c is computed from buffer c % 2 while channel c + 1 is fetched;
  // unrolled by two so that the buffer offsets are constants
  fetch(0);
  put(0);
  __syncthreads();
  // (past the last channel the last one is fetched again, unused)
  const uint32_t last = cin - 1;
  for (uint32_t c = 0; c < cin; c += 2) {
    fetch(min(c + 1, last));
    compute(0, c);
    put(1);
    __syncthreads();
    if (c + 1 == cin) break;
    fetch(min(c + 2, last));
    compute(1, c + 1);
    put(0);
    __syncthreads();
  }
  const uint32_t py = ty0 + ty, px = tx0 + tx;
  if (py < ph && px < pw) {
#pragma unroll
    for (int k = 0; k < OC; ++k) {
      const double m = fmax(fmax(acc[k][0], acc[k][1]), fmax(acc[k][2], acc[k][3]));
      y[(static_cast<uint64_t>(o0 + k) * ph + py) * pw + px] = static_cast<float>(fmax(m, 0.0));
    }
  }
}

// The same convolution as an implicit GEMM on the fp64 matrix cores
// (v_mfma_f64_16x16x4f64: D[16x16] += A[16x4] * B[4x16], lane l supplying
// A[l % 16][l / 16] and B[l / 16][l % 16] and holding D[4 r + l / 16][l % 16]
// in its r-th result, as an in-bounds probe of the instruction showed).  Rows of the product are convolution outputs, columns
// output channels, and the reduction runs over (tap, input channel) pairs
// k = tap * cin + c, so that a lane's four consecutive k of one MFMA are four
// input channels of one tap and every operand address is the lane's base plus
// a uniform offset.  A workgroup of four waves computes a 16 x 16 tile of
// convolution outputs (8 x 8 pooled) for 16 * NJB output channels: each wave
// four 4 x 4 pixel blocks (one MFMA row each: row i = pixel (i / 4, i % 4)),
// so per reduction step it reads four A and NJB B values and issues 4 NJB
// independent MFMAs.  The input tile (cin x 18 x 18, zero padded) and the
// weights ([k][channel], fp32) are staged in LDS four input channels at a
// time, the next four channels' loads in flight while the current ones'
// products run.  Bias is
// the accumulator's start; after the reduction a lane holds one pixel column
// (px = l / 16, rows py = r) of a block for one channel, so the 2 x 2 pooling
// is a max inside the lane (rows) and one across lanes l and l ^ 16
// (columns), then ReLU (monotone, so it commutes with the max).  Needs cin % 4 == 0, cout % 16 == 0 and the staged tile and
// weights within 64 KB of LDS (conv_mfma_lds).
typedef double double4_t __attribute__((ext_vector_type(4)));
constexpr int kConvMfmaTile = 16;                      // convolution outputs per tile side
constexpr int kConvMfmaIn = kConvMfmaTile + 2;         // 18 staged rows / columns
constexpr size_t kConvMfmaMaxLds = 64 * 1024;

template <int NJB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_conv3x3_relu_pool_mfma(
    const float* __restrict__ x, const float* __restrict__ w, const float* __restrict__ bias, float* __restrict__ y,
    uint32_t cin, uint32_t h, uint32_t wd, uint32_t tiles_x) {
  constexpr int NC = 16 * NJB;                         // output channels of this workgroup
  constexpr int kPlane = kConvMfmaIn * kConvMfmaIn;    // 324
  constexpr int kOut = kConvMfmaTile / 2;              // 8 x 8 pooled outputs per channel
  // One group = four input channels, the channels of one reduction step per
  // tap: its input tile (4 x 324) and its weights (9 taps x 4 x NC) take
  // kInSlots and kWSlots elements per thread.
  constexpr int kInSlots = (4 * kPlane + 255) / 256;
  constexpr int kWSlots = (9 * 4 * NC + 255) / 256;
  extern __shared__ float s_dyn[];
  float* s_in = s_dyn;                                 // [cin][18][18]
  float* s_w = s_dyn + cin * kPlane;                   // [9 cin][NC], row k = tap * cin + c
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Y0 = static_cast<int>((blockIdx.x / tiles_x) * kConvMfmaTile);
  const int X0 = static_cast<int>((blockIdx.x % tiles_x) * kConvMfmaTile);
  const uint32_t o0 = blockIdx.y * NC;
  const uint64_t plane = static_cast<uint64_t>(h) * wd;
  // this thread's input elements of a group (fixed positions; zero padding
  // outside the image)
  uint32_t ioff[kInSlots];
  uint32_t imask = 0;
#pragma unroll
  for (int j = 0; j < kInSlots; ++j) {
    const uint32_t e = tid + 256 * j, cl = e / kPlane, rq = e % kPlane;
    const int gy = Y0 - 1 + static_cast<int>(rq / kConvMfmaIn), gx = X0 - 1 + static_cast<int>(rq % kConvMfmaIn);
    const bool in = e < 4 * kPlane && gy >= 0 && gy < static_cast<int>(h) && gx >= 0 && gx < static_cast<int>(wd);
    ioff[j] = in ? cl * static_cast<uint32_t>(plane) + static_cast<uint32_t>(gy) * wd + static_cast<uint32_t>(gx) : 0u;
    imask |= (in ? 1u : 0u) << j;
  }
  // Group g's loads go to registers (vi, vw) and from there to LDS, so the
  // next group's loads are in flight while this group's products run.
  // Weight element e of a group: channel jj = e % NC (lanes over output
  // channels, so the LDS stores hit consecutive banks), then tap and channel.
  float vi[kInSlots], vw[kWSlots];
  auto fetch = [&](uint32_t g) {
    const float* xg = x + static_cast<uint64_t>(4 * g) * plane;
#pragma unroll
    for (int j = 0; j < kInSlots; ++j) vi[j] = ((imask >> j) & 1u) ? xg[ioff[j]] : 0.0f;
#pragma unroll
    for (int j = 0; j < kWSlots; ++j) {
      const uint32_t e = tid + 256 * j, jj = e % NC, rem = e / NC, t = rem % 9, cl = rem / 9;
      vw[j] = e < 9 * 4 * NC ? w[(static_cast<uint64_t>(o0 + jj) * cin + 4 * g + cl) * 9 + t] : 0.0f;
    }
  };
  auto put = [&](uint32_t g) {
#pragma unroll
    for (int j = 0; j < kInSlots; ++j) {
      const uint32_t e = tid + 256 * j;
      if (e < 4 * kPlane) s_in[4 * g * kPlane + e] = vi[j];
    }
#pragma unroll
    for (int j = 0; j < kWSlots; ++j) {
      const uint32_t e = tid + 256 * j, jj = e % NC, rem = e / NC, t = rem % 9, cl = rem / 9;
      if (e < 9 * 4 * NC) s_w[(t * cin + 4 * g + cl) * NC + jj] = vw[j];
    }
  };
  // lane roles: A row i = pixel (py, px) of a 4 x 4 block, reduction slot kq
  const uint32_t i = lane & 15, kq = lane >> 4, py = i >> 2, px = i & 3;
  // this wave's four blocks: block row `wave` of the tile, block columns 0..3
  const float* a_base = s_in + kq * kPlane + (4 * wave + py) * kConvMfmaIn + px;
  const float* b_base = s_w + kq * NC + i;
  double4_t acc[4][NJB];
#pragma unroll
  for (int jb = 0; jb < NJB; ++jb) {
    const double b0 = static_cast<double>(bias[o0 + 16 * jb + i]);
#pragma unroll
    for (int bx = 0; bx < 4; ++bx) acc[bx][jb] = double4_t{b0, b0, b0, b0};
  }
  const uint32_t ng = cin / 4;
  fetch(0);
  put(0);
  __syncthreads();
  for (uint32_t g = 0; g < ng; ++g) {
    if (g + 1 < ng) fetch(g + 1);
    const float* ag = a_base + 4 * g * kPlane;
    const float* bg = b_base + 4 * g * NC;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      const float* ap = ag + dy * kConvMfmaIn + dx;
      const float* bp = bg + t * cin * NC;
      double bv[NJB];
#pragma unroll
      for (int jb = 0; jb < NJB; ++jb) bv[jb] = static_cast<double>(bp[16 * jb]);
#pragma unroll
      for (int bx = 0; bx < 4; ++bx) {
        const double av = static_cast<double>(ap[4 * bx]);
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb)
          acc[bx][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[jb], acc[bx][jb], 0, 0, 0);
      }
    }
    if (g + 1 < ng) put(g + 1);
    __syncthreads();
  }
  // Pooling: this lane holds pixel column px = kq of each block, rows 0..3
  // in its four results; pooled row 0 from rows 0-1, row 1 from rows 2-3.
  // The pooled tile [NC][8][8] goes through LDS (over the input tile, which
  // every wave has finished reading at the last barrier) so that each of its
  // rows is written as 32 contiguous bytes.
  float* s_out = s_dyn;
#pragma unroll
  for (int jb = 0; jb < NJB; ++jb) {
#pragma unroll
    for (int bx = 0; bx < 4; ++bx) {
      double m0 = fmax(acc[bx][jb][0], acc[bx][jb][1]);
      double m1 = fmax(acc[bx][jb][2], acc[bx][jb][3]);
      m0 = fmax(m0, __shfl_xor(m0, 16));
      m1 = fmax(m1, __shfl_xor(m1, 16));
      if ((kq & 1) == 0) {
        float* o = s_out + ((16 * jb + i) * kOut + 2 * wave) * kOut + 2 * bx + (kq >> 1);
        o[0] = static_cast<float>(fmax(m0, 0.0));
        o[kOut] = static_cast<float>(fmax(m1, 0.0));
      }
    }
  }
  __syncthreads();
  const uint32_t ph = h / 2, pw = wd / 2, PY0 = static_cast<uint32_t>(Y0 / 2), PX0 = static_cast<uint32_t>(X0 / 2);
  for (uint32_t rrow = tid; rrow < NC * kOut; rrow += 256) {
    const uint32_t ch = rrow / kOut, ry = rrow % kOut, PY = PY0 + ry;
    if (PY >= ph) continue;
    const float* src = s_out + rrow * kOut;
    float* dst = y + (static_cast<uint64_t>(o0 + ch) * ph + PY) * pw + PX0;
    if (PX0 + kOut <= pw && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
      reinterpret_cast<float4*>(dst)[0] = reinterpret_cast<const float4*>(src)[0];
      reinterpret_cast<float4*>(dst)[1] = reinterpret_cast<const float4*>(src)[1];
    } else {
      for (uint32_t k = 0; k < kOut && PX0 + k < pw; ++k) dst[k] = src[k];
    }
  }
}

size_t conv_mfma_lds(uint32_t cin, uint32_t njb) {
  // the staged input tile and weights; the pooled tile [16 njb][8][8] reuses it
  const size_t staged = 4 * (static_cast<size_t>(cin) * kConvMfmaIn * kConvMfmaIn + 9ull * cin * 16 * njb);
  return std::max<size_t>(staged, 4ull * 16 * njb * 64);
}
// Output-channel blocks of 16 per workgroup for the matrix-core form (2 where
// cout allows and the LDS fits, else 1); 0 = the form does not apply.
uint32_t conv_mfma_njb(uint32_t cin, uint32_t cout) {
  if (cin % 4 != 0 || cout % 16 != 0) return 0;
  if (cout % 32 == 0 && conv_mfma_lds(cin, 2) <= kConvMfmaMaxLds) return 2;
  return conv_mfma_lds(cin, 1) <= kConvMfmaMaxLds ? 1 : 0;
}

// fp64 copy of convolution weights for the scalar-weight variant:
// w64[(c * cout + o) * 9 + t] = w[(o * cin + c) * 9 + t] (exact conversion).
__global__ __launch_bounds__(256) void k_conv_weights_f64(const float* __restrict__ w, double* __restrict__ w64,
                                                          uint32_t cin, uint32_t cout) {
  const uint64_t n = static_cast<uint64_t>(cin) * cout * 9;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += 256ull * gridDim.x) {
    const uint64_t t = i % 9, oc = i / 9;
    const uint64_t o = oc % cout, c = oc / cout;
    w64[i] = static_cast<double>(w[(o * cin + c) * 9 + t]);
  }
}

// y = W x + b for M <= 16 outputs of a long input: every workgroup sums its
// grid-stride share of the inputs for all M outputs (fp64), reduces them in
// a fixed order and publishes M partials; the last workgroup to finish adds
// the partials in workgroup order and the bias.
constexpr int kDenseMaxOut = 16;

// Second half of the dense layer: sh[w * 16 + j] holds wave w's sum for
// output j.  The block adds its waves in order and publishes M partials; the
// last block to arrive adds all partials in block order, plus the bias.
template <int M>
__device__ void dense_finish(double* sh, int* flag, const float* __restrict__ bias, float* __restrict__ y,
                             uint32_t* counter, uint64_t* partials) {
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (threadIdx.x < M) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += sh[q * kDenseMaxOut + threadIdx.x];
    __hip_atomic_store(&partials[static_cast<uint64_t>(blockIdx.x) * kDenseMaxOut + threadIdx.x], d2u(t),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  if (arrive_last(counter, flag)) {
    // thread t adds, in block order, the partials of output t % 16 over one
    // contiguous range of blocks (range t / 16), eight agent-scope loads in
    // flight at a time (each is a trip past the L2, so loading them one
    // after another would cost a full latency apiece); the ranges are then
    // added in order
    const uint32_t j = threadIdx.x % kDenseMaxOut, r = threadIdx.x / kDenseMaxOut;
    const uint32_t nr = blockDim.x / kDenseMaxOut;
    const uint32_t per = (gridDim.x + nr - 1) / nr;
    const uint32_t q1 = min((r + 1) * per, gridDim.x);
    uint32_t q = min(r * per, gridDim.x);
    double t = 0.0;
    if (j < static_cast<uint32_t>(M)) {
      for (; q + 8 <= q1; q += 8) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = read_partial(partials, (q + u) * kDenseMaxOut + j);
#pragma unroll
        for (int u = 0; u < 8; ++u) t += u2d(v[u]);
      }
      for (; q < q1; ++q) t += u2d(read_partial(partials, q * kDenseMaxOut + j));
    }
    sh[r * kDenseMaxOut + j] = t;
    __syncthreads();
    if (threadIdx.x < M) {
      double sum = 0.0;
      for (uint32_t k = 0; k < nr; ++k) sum += sh[k * kDenseMaxOut + threadIdx.x];
      y[threadIdx.x] = static_cast<float>(sum + static_cast<double>(bias[threadIdx.x]));
    }
    reset_counter(counter);
  }
}

// W is stored input-major (n x M: the M weights of input i are adjacent), so
// a wave streams 64 consecutive inputs' weights, M * 256 contiguous bytes,
// with 16-byte loads when M is a multiple of 4 and W is 16-byte aligned
// (vec).  M is a template parameter: the loads of a row are issued without
// branches between them.
template <int M>
__global__ __launch_bounds__(1024) void k_dense(const float* __restrict__ x, const float* __restrict__ W,
                                                const float* __restrict__ bias, float* __restrict__ y, uint64_t n,
                                                int vec, uint32_t* counter, uint64_t* partials) {
  __shared__ double sh[1024];  // 16 waves x 16 outputs, then 64 ranges x 16 outputs
  __shared__ int flag;
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  double acc[M];
#pragma unroll
  for (int j = 0; j < M; ++j) acc[j] = 0.0;
  if constexpr (M % 4 == 0) {
    if (vec) {
      for (uint64_t i = gid; i < n; i += stride) {
        const double xi = static_cast<double>(x[i]);
        const float4* wr = reinterpret_cast<const float4*>(W + i * M);
        float4 v[M / 4];
#pragma unroll
        for (int q = 0; q < M / 4; ++q) v[q] = wr[q];
#pragma unroll
        for (int q = 0; q < M / 4; ++q) {
          acc[4 * q] = fma(static_cast<double>(v[q].x), xi, acc[4 * q]);
          acc[4 * q + 1] = fma(static_cast<double>(v[q].y), xi, acc[4 * q + 1]);
          acc[4 * q + 2] = fma(static_cast<double>(v[q].z), xi, acc[4 * q + 2]);
          acc[4 * q + 3] = fma(static_cast<double>(v[q].w), xi, acc[4 * q + 3]);
        }
      }
    }
  }
  if (M % 4 != 0 || !vec) {
    for (uint64_t i = gid; i < n; i += stride) {
      const double xi = static_cast<double>(x[i]);
#pragma unroll
      for (int j = 0; j < M; ++j) acc[j] = fma(static_cast<double>(W[i * M + j]), xi, acc[j]);
    }
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wv_ = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double t = wave_sum(acc[j]);
    if (lane == 0) sh[wv_ * kDenseMaxOut + j] = t;
  }
  dense_finish<M>(sh, &flag, bias, y, counter, partials);
}

// Variants 1 and 2, for M in {4, 8, 16} and 16-byte aligned W: a wave takes 64
// inputs at a time (a chunk) and reads their weights, M * 256 bytes, as M / 4
// fully contiguous 1 KB loads; lane l then always holds the four outputs
// 4l % M .. 4l % M + 3, of inputs (256 q + 4 l) / M of the chunk.  U (2 or
// 4) chunks are loaded before any is used.  At the end the lanes holding the
// same outputs are added by a fixed butterfly (masks M/4 .. 32), so the sum
// order is fixed for a given launch shape.
//
// SPLIT: the blocks only store their partials, and a second one-block kernel
// on the same stream adds them (no ticket counter, no fences): each block's
// agent-scope release fence and ticket atomic cost ~40 ns, serialised over
// the blocks, which is ~11 us at 256 blocks.
template <int M, int U, bool SPLIT>
__global__ __launch_bounds__(1024) void k_dense_lanes(const float* __restrict__ x, const float* __restrict__ W,
                                                      const float* __restrict__ bias, float* __restrict__ y,
                                                      uint64_t n, uint32_t* counter, uint64_t* partials) {
  static_assert(M == 4 || M == 8 || M == 16, "outputs must divide the 256 floats of a 1 KB load");
  constexpr int kQ = M / 4;  // 1 KB loads per chunk
  constexpr int kU = U;      // chunks in flight per lane
  __shared__ double sh[1024];  // 16 waves x 16 outputs, then 64 ranges x 16 outputs
  __shared__ int flag;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * blockDim.x / kWave;
  const uint64_t chunks = n / kWave;
  const float4* W4 = reinterpret_cast<const float4*>(W);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto add = [&](const float4& v, float xf) {
    const double xi = static_cast<double>(xf);
    acc[0] = fma(static_cast<double>(v.x), xi, acc[0]);
    acc[1] = fma(static_cast<double>(v.y), xi, acc[1]);
    acc[2] = fma(static_cast<double>(v.z), xi, acc[2]);
    acc[3] = fma(static_cast<double>(v.w), xi, acc[3]);
  };
  uint64_t c = wave;
  for (; c + (kU - 1) * nwaves < chunks; c += kU * nwaves) {
    float4 v[kU][kQ];
    float xv[kU][kQ];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const uint64_t cc = c + u * nwaves;
        v[u][q] = W4[cc * (kWave * kQ) + q * kWave + lane];
        xv[u][q] = x[cc * kWave + (256u * q + 4u * lane) / M];
      }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int q = 0; q < kQ; ++q) add(v[u][q], xv[u][q]);
  }
  for (; c < chunks; c += nwaves) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) add(W4[c * (kWave * kQ) + q * kWave + lane], x[c * kWave + (256u * q + 4u * lane) / M]);
  }
  // the partial chunk of the last n % 64 inputs: the wave whose turn it is
  if (c == chunks) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const uint64_t i = c * kWave + (256u * q + 4u * lane) / M;
      if (i < n) add(W4[c * (kWave * kQ) + q * kWave + lane], x[i]);
    }
  }
#pragma unroll
  for (int mask = kQ; mask < kWave; mask <<= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += __shfl_xor(acc[k], mask, kWave);
  if (lane < static_cast<uint32_t>(kQ)) {
    const int wv_ = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[wv_ * kDenseMaxOut + 4 * lane + k] = acc[k];
  }
  if constexpr (SPLIT) {
    __syncthreads();
    if (threadIdx.x < M) {
      const int nw = (blockDim.x + kWave - 1) / kWave;
      double t = 0.0;
      for (int q = 0; q < nw; ++q) t += sh[q * kDenseMaxOut + threadIdx.x];
      partials[static_cast<uint64_t>(blockIdx.x) * kDenseMaxOut + threadIdx.x] = d2u(t);
    }
  } else {
    dense_finish<M>(sh, &flag, bias, y, counter, partials);
  }
}

// Final step of the split dense layer: one workgroup adds the partials of
// nblocks blocks in the order of dense_finish (output j = t % 16 over one
// range of blocks per thread, then the ranges in order), plus the bias.
template <int M>
__global__ __launch_bounds__(1024) void k_dense_final(const uint64_t* __restrict__ partials, uint32_t nblocks,
                                                      const float* __restrict__ bias, float* __restrict__ y) {
  __shared__ double sh[1024];
  const uint32_t j = threadIdx.x % kDenseMaxOut, r = threadIdx.x / kDenseMaxOut;
  const uint32_t nr = blockDim.x / kDenseMaxOut;
  const uint32_t per = (nblocks + nr - 1) / nr;
  const uint32_t q1 = min((r + 1) * per, nblocks);
  double t = 0.0;
  if (j < static_cast<uint32_t>(M)) {
    // eight loads in flight, then added in block order
    uint32_t q = min(r * per, nblocks);
    for (; q + 8 <= q1; q += 8) {
      uint64_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partials[(q + u) * kDenseMaxOut + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) t += u2d(v[u]);
    }
    for (; q < q1; ++q) t += u2d(partials[q * kDenseMaxOut + j]);
  }
  sh[r * kDenseMaxOut + j] = t;
  __syncthreads();
  if (threadIdx.x < M) {
    double sum = 0.0;
    for (uint32_t k = 0; k < nr; ++k) sum += sh[k * kDenseMaxOut + threadIdx.x];
    y[threadIdx.x] = static_cast<float>(sum + static_cast<double>(bias[threadIdx.x]));
  }
}

// p = sigmoid(w . [e1; e2] + b), 2m <= 64: one wave, a fixed butterfly sum.
__global__ __launch_bounds__(64) void k_siamese_combine(const float* __restrict__ e1, const float* __restrict__ e2,
                                                        const float* __restrict__ w, const float* __restrict__ b,
                                                        float* __restrict__ p, uint32_t m) {
  const uint32_t k = threadIdx.x;
  double t = 0.0;
  if (k < 2 * m) t = static_cast<double>(w[k]) * static_cast<double>(k < m ? e1[k] : e2[k - m]);
  const double s = wave_sum(t) + static_cast<double>(b[0]);
  if (k == 0) p[0] = static_cast<float>(1.0 / (1.0 + exp(-s)));
}

// ---------------------------------------------------------------------------
// Utilities: a delay kernel for scheduler tests and a plain copy.
// ---------------------------------------------------------------------------
__global__ void k_spin(uint64_t ticks) {
  if (threadIdx.x == 0) {
    const uint64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
  }
}

// Last node of a captured region graph: each workgroup makes a system-scope
// release, which writes back every dirty line of its XCD's L2 to memory, so
// what the graph's kernels stored is visible to the copy engines and to the
// host once the graph's completion is signalled.  Workgroups are handed to
// the eight XCDs round-robin by id, so 64 of them reach every L2.
__global__ __launch_bounds__(64) void k_release_l2() { __threadfence_system(); }

// Completion signals between streams.  A task's signal is one word per
// stream that a one-wave kernel, queued right after the task on its stream,
// raises to the task's sequence number there: the task has finished (and its
// end-of-kernel release has been made) before that kernel runs, because the
// stream runs its work in order.  A consumer on another stream is queued
// behind a one-wave kernel that polls the words it needs until each reaches
// its value; the consumer's own dispatch, ordered after that kernel, makes the
// acquire that makes the producer's stores visible to it.  Polls use
// device-coherent atomic loads and sleep between tries; past max_ticks of the
// constant-rate clock the poller gives up, raises the flag in host memory and
// exits, so every wave ends.
__global__ __launch_bounds__(64) void k_dag_signal(uint64_t* word, uint64_t value) {
  if (threadIdx.x == 0) __hip_atomic_store(word, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(64) void k_dag_wait(SignalWaits w) {
  if (threadIdx.x != 0) return;
  const uint64_t t0 = wall_clock64();
  for (uint32_t i = 0; i < w.n; ++i) {
    const uint64_t* word = w.words + static_cast<uint64_t>(w.slot[i]) * kSignalStride;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < w.value[i]) {
      if (wall_clock64() - t0 > w.max_ticks) {
        __hip_atomic_store(w.timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

// Host<->device copy by the CUs (pinned host memory is read or written over
// PCIe by the kernel itself): 16-byte words when both ends are 16-byte
// aligned, then the tail bytes.
__global__ __launch_bounds__(256) void k_copy_bytes(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                    uint64_t n) {
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 == 0) {
    const uint64_t n16 = n / 16;
    for (uint64_t i = gid; i < n16; i += stride)
      reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    done = n16 * 16;
  }
  for (uint64_t i = done + gid; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(1024) void k_copy_f32(const float* __restrict__ src,
                                                   float* __restrict__ dst, uint64_t n, int vec) {
  const uint64_t gid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t start = 0;
  if (vec) {
    const uint64_t n4 = n >> 2;
    for (uint64_t i = gid; i < n4; i += stride)
      reinterpret_cast<float4*>(dst)[i] = reinterpret_cast<const float4*>(src)[i];
    start = n4 << 2;
  }
  for (uint64_t i = start + gid; i < n; i += stride) dst[i] = src[i];
}

// ===========================================================================
// Host side: argument checks and launches
// ===========================================================================
const char* cfg_block_any(const LaunchCfg& c) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be a multiple of 64 in [64, 1024]";
  if (c.variant != 0) return "variant must be 0";
  return nullptr;
}
const char* cfg_bs(const LaunchCfg& c) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be a multiple of 64 in [64, 1024]";
  if (c.variant > 2)
    return "variant: 0 = library erfc, 1 = one exponential and one polynomial per CDF, 2 = 1 with own log/exp";
  return nullptr;
}
const char* cfg_reduce(const LaunchCfg& c) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be a multiple of 64 in [64, 1024]";
  if (c.variant > 1) return "variant: 0 = two kernels, 1 = single pass";
  return nullptr;
}
const char* cfg_tile(const LaunchCfg& c);
const char* cfg_spmv(const LaunchCfg& c) {
  if (c.block != 256) return "SpMV runs 256-thread workgroups";
  if (c.grid_cap != 0 && (c.variant & 0x500u) != 0x500u)
    return "grid_cap must be 0 (it caps the workgroups of the resident row-window variants 0x504 and 0x508)";
  const uint32_t ipt = c.variant & 0xffu;
  if (c.variant & 0x100u) {
    const uint32_t mode = c.variant & 0x600u;
    if (c.variant > 0x7ffu || (ipt != 4 && ipt != 8 && ipt != 16) || mode == 0x600u || (mode == 0x400u && ipt == 16))
      return "row-window SpMV variant must be 0x100 | 4, 8 or 16 (nonzeros per thread), plus 0x200 for "
             "streaming loads of the matrix or 0x400 (4 or 8 per thread) for a resident grid that loads each "
             "workgroup's next tile early";
    return nullptr;
  }
  if (c.variant != 4 && c.variant != 8 && c.variant != 12 && c.variant != 16)
    return "SpMV variant must be 4, 8, 12 or 16 (merge-path items per thread) or 0x100 | 4, 8 or 16 "
           "(row windows)";
  return nullptr;
}
const char* cfg_spin(const LaunchCfg& c) {
  if (c.block != 64 || c.grid_cap != 0 || c.variant != 0) return "spin runs one 64-thread workgroup";
  return nullptr;
}

uint32_t stream_grid(uint64_t work, const LaunchCfg& c) {
  uint64_t g = ceil_div(std::max<uint64_t>(work, 1), c.block);
  if (c.grid_cap) g = std::min<uint64_t>(g, c.grid_cap);
  return static_cast<uint32_t>(std::max<uint64_t>(std::min<uint64_t>(g, 1u << 30), 1));
}

uint64_t reduction_capacity(size_t scratch_bytes) {
  return scratch_bytes > kScratchPartialsOffset ? (scratch_bytes - kScratchPartialsOffset) / 8 : 0;
}

uint32_t reduction_grid(uint64_t work, const LaunchCfg& c, size_t scratch_bytes) {
  uint64_t g = stream_grid(work, c);
  g = std::min<uint64_t>(g, reduction_capacity(scratch_bytes));
  return static_cast<uint32_t>(std::max<uint64_t>(g, 1));
}

uint64_t pn(const void* p) { return static_cast<const dag_p_n*>(p)->n; }

bool mul_fits(uint64_t a, uint64_t b, size_t have) {
  return a <= (~0ull) / b && a * b <= have;
}

// -- VEC --------------------------------------------------------------------
const char* v_vec_square(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  return mul_fits(pn(p), 4, sz[0]) ? nullptr : "x smaller than 4*n bytes";
}
hipError_t l_vec_square(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const uint64_t n = pn(p);
  if (n == 0) return hipSuccess;
  const int vec = aligned16(a[0]);
  DAGRT_LAUNCH(k_vec_square, dim3(stream_grid(vec ? ceil_div(n, 4) : n, c)), dim3(c.block), 0, s,
                     static_cast<float*>(a[0]), n, vec);
  return hipGetLastError();
}

const char* v_vec_sum_diff(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t sb) {
  const uint64_t n = pn(p);
  if (!mul_fits(n, 4, sz[0]) || !mul_fits(n, 4, sz[1])) return "x or y smaller than 4*n bytes";
  if (sz[2] < 4) return "r smaller than 4 bytes";
  if (reduction_capacity(sb) < 1) return "scratch too small";
  return nullptr;
}
hipError_t l_vec_sum_diff(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t sb) {
  const uint64_t n = pn(p);
  const int vec = aligned16(a[0]) && aligned16(a[1]);
  auto* counter = static_cast<uint32_t*>(scr);
  auto* partials = reinterpret_cast<uint64_t*>(static_cast<char*>(scr) + kScratchPartialsOffset);
  const uint32_t g = reduction_grid(vec ? ceil_div(n, 4) : n, c, sb);
  if (c.variant == 1) {
    DAGRT_LAUNCH(k_vec_sum_diff<true>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                       static_cast<const float*>(a[1]), static_cast<float*>(a[2]), n, vec, counter, partials);
    return hipGetLastError();
  }
  DAGRT_LAUNCH(k_vec_sum_diff<false>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                     static_cast<const float*>(a[1]), static_cast<float*>(a[2]), n, vec, counter, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DAGRT_LAUNCH(k_finish_sum<float>, dim3(1), dim3(256), 0, s, partials, g, static_cast<float*>(a[2]));
  return hipGetLastError();
}

// -- B&S --------------------------------------------------------------------
const char* v_bs(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const auto* q = static_cast<const dag_p_bs*>(p);
  if (!mul_fits(q->n, 4, sz[0]) || !mul_fits(q->n, 4, sz[1])) return "S or C smaller than 4*n bytes";
  if (!(q->strike > 0) || !(q->vol > 0) || !(q->years > 0)) return "strike, vol and years must be > 0";
  return nullptr;
}
hipError_t l_bs(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const auto* q = static_cast<const dag_p_bs*>(p);
  if (q->n == 0) return hipSuccess;
  BsConst k;
  k.strike = q->strike;
  k.vol_t = q->vol * std::sqrt(q->years);
  k.mu_t = (q->rate + 0.5 * q->vol * q->vol) * q->years;
  k.disc_strike = q->strike * std::exp(-q->rate * q->years);
  k.inv_strike = 1.0 / q->strike;
  k.inv_vol_t = 1.0 / k.vol_t;
  k.growth = std::exp(q->rate * q->years) / q->strike;
  const int vec = aligned16(a[0]) && aligned16(a[1]);
  const dim3 grid(stream_grid(vec ? ceil_div(q->n, 4) : q->n, c));
  if (c.variant == 1) {
    DAGRT_LAUNCH(k_bs_call<1>, grid, dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                 static_cast<float*>(a[1]), q->n, vec, k);
  } else if (c.variant == 2) {
    DAGRT_LAUNCH(k_bs_call<2>, grid, dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                 static_cast<float*>(a[1]), q->n, vec, k);
  } else {
    DAGRT_LAUNCH(k_bs_call<0>, grid, dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                 static_cast<float*>(a[1]), q->n, vec, k);
  }
  return hipGetLastError();
}

// -- IMG --------------------------------------------------------------------
const char* v_img2(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const auto* q = static_cast<const dag_p_img*>(p);
  if (q->w == 0 || q->h == 0) return "empty image";
  const uint64_t n = static_cast<uint64_t>(q->w) * q->h;
  if (n > (1ull << 31)) return "image larger than 2^31 pixels";
  if (!mul_fits(n, 4, sz[0]) || !mul_fits(n, 4, sz[1])) return "image buffers smaller than 4*w*h bytes";
  return nullptr;
}
const char* v_blur(const void* p, const size_t* sz, uint32_t na, const LaunchCfg& c, size_t sb) {
  const auto* q = static_cast<const dag_p_img*>(p);
  if (q->ksize < 1 || q->ksize > 31 || q->ksize % 2 == 0) return "ksize must be odd in [1, 31]";
  return v_img2(p, sz, na, c, sb);
}

// Tile shapes of the stencils (launch variant >> 1) and their workgroup sizes.
struct TileShape {
  int tw, th;
};
constexpr TileShape kTileShapes[] = {{64, 16}, {64, 8}, {64, 4}, {32, 8}};
constexpr uint32_t kNumTileShapes = sizeof(kTileShapes) / sizeof(kTileShapes[0]);

// Variant bit 3: resident grid with the next tile's loads in flight, for the
// 64-wide shapes with the per-XCD tile order (variants 9 and 11).
constexpr uint32_t kTileResident = 8;

const char* cfg_tile(const LaunchCfg& c) {
  if (c.grid_cap != 0 && !(c.variant & kTileResident))
    return "grid_cap must be 0 (it caps the workgroups of the resident variants only)";
  const uint32_t shape = (c.variant & ~kTileResident) >> 1;
  if (shape >= kNumTileShapes || ((c.variant & kTileResident) && c.variant != 9 && c.variant != 11))
    return "variant: bit 0 = tile order (0 row-major, 1 one contiguous run of tiles per XCD), "
           "bits 1-2 = tile shape (0: 64x16, 1: 64x8, 2: 64x4, 3: 32x8), bit 3 = resident grid loading each "
           "workgroup's next tile early (9: 64x16, 11: 64x8)";
  const TileShape t = kTileShapes[shape];
  if (c.block != static_cast<uint32_t>(t.tw * t.th / kRowsPerThread))
    return "block must be the tile's threads: 256 for 64x16, 128 for 64x8, 64 for 64x4 and 32x8";
  return nullptr;
}

template <int R, int TW, int TH>
void launch_blur_shape(hipStream_t s, const float* in, float* out, int w, int h, const GaussW& wt, int xcd_map) {
  const int tx = static_cast<int>(ceil_div(w, TW)), nt = tx * static_cast<int>(ceil_div(h, TH));
  const int grid = xcd_map ? 8 * ((nt + 7) / 8) : nt;
  DAGRT_LAUNCH((k_gauss_blur<R, TW, TH>), dim3(grid), dim3(TW * TH / kRowsPerThread), 0, s, in, out, w, h, wt, tx,
               nt, xcd_map);
}

// Compute units of the current device (cached per device ordinal).
int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Workgroups of a resident tile grid: as many as fit on the GPU at once
// (occupancy of the kernel, asked once per instantiation through *per_cu)
// or cap if that is smaller (0: no cap), a multiple of 8 so that every XCD
// gets the same count, at most one per tile.
int resident_tile_grid(const void* kern, int threads, int ntiles, int* per_cu, uint32_t cap) {
  if (*per_cu == 0) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, 0);
    *per_cu = (e == hipSuccess && n > 0) ? n : 2;
  }
  int per_xcd = std::min((ntiles + 7) / 8, *per_cu * device_cus() / 8);
  if (cap) per_xcd = std::min<int64_t>(per_xcd, cap / 8);
  return 8 * std::max(1, per_xcd);
}

template <int R, int TH>
void launch_blur_rt(hipStream_t s, const float* in, float* out, int w, int h, const GaussW& wt, uint32_t cap) {
  static int per_cu = 0;
  const int tx = static_cast<int>(ceil_div(w, 64)), nt = tx * static_cast<int>(ceil_div(h, TH));
  const int grid = resident_tile_grid(reinterpret_cast<const void*>(&k_gauss_blur_rt<R, TH>),
                                      64 * TH / kRowsPerThread, nt, &per_cu, cap);
  DAGRT_LAUNCH((k_gauss_blur_rt<R, TH>), dim3(grid), dim3(64 * TH / kRowsPerThread), 0, s, in, out, w, h, wt,
               tx, nt);
}

template <int R>
void launch_blur_r(hipStream_t s, const float* in, float* out, int w, int h, const GaussW& wt, uint32_t variant,
                   uint32_t cap) {
  const int xm = static_cast<int>(variant & 1);
  if (variant == 9) return launch_blur_rt<R, 16>(s, in, out, w, h, wt, cap);
  if (variant == 11) return launch_blur_rt<R, 8>(s, in, out, w, h, wt, cap);
  switch (variant >> 1) {
    case 1: launch_blur_shape<R, 64, 8>(s, in, out, w, h, wt, xm); break;
    case 2: launch_blur_shape<R, 64, 4>(s, in, out, w, h, wt, xm); break;
    case 3: launch_blur_shape<R, 32, 8>(s, in, out, w, h, wt, xm); break;
    default: launch_blur_shape<R, 64, 16>(s, in, out, w, h, wt, xm); break;
  }
}

hipError_t l_blur(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const auto* q = static_cast<const dag_p_img*>(p);
  const uint32_t vr = c.variant;
  const int k = static_cast<int>(q->ksize), rad = (k - 1) / 2;
  const double sigma = k / 6.0;
  GaussW wt{};
  double sum = 0.0;
  for (int i = -rad; i <= rad; ++i) {
    wt.w[i + rad] = std::exp(-(static_cast<double>(i) * i) / (2.0 * sigma * sigma));
    sum += wt.w[i + rad];
  }
  for (int i = 0; i < k; ++i) wt.w[i] /= sum;
  const auto* in = static_cast<const float*>(a[0]);
  auto* out = static_cast<float*>(a[1]);
  const int w = static_cast<int>(q->w), h = static_cast<int>(q->h);
  switch (rad) {
    case 0: launch_blur_r<0>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 1: launch_blur_r<1>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 2: launch_blur_r<2>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 3: launch_blur_r<3>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 4: launch_blur_r<4>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 5: launch_blur_r<5>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 6: launch_blur_r<6>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 7: launch_blur_r<7>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 8: launch_blur_r<8>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 9: launch_blur_r<9>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 10: launch_blur_r<10>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 11: launch_blur_r<11>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 12: launch_blur_r<12>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 13: launch_blur_r<13>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    case 14: launch_blur_r<14>(s, in, out, w, h, wt, vr, c.grid_cap); break;
    default: launch_blur_r<15>(s, in, out, w, h, wt, vr, c.grid_cap); break;
  }
  return hipGetLastError();
}

template <int TW, int TH>
void launch_sobel_shape(hipStream_t s, const float* in, float* out, int w, int h, int xcd_map) {
  const int tx = static_cast<int>(ceil_div(w, TW)), nt = tx * static_cast<int>(ceil_div(h, TH));
  const int grid = xcd_map ? 8 * ((nt + 7) / 8) : nt;
  DAGRT_LAUNCH((k_sobel<TW, TH>), dim3(grid), dim3(TW * TH / kRowsPerThread), 0, s, in, out, w, h, tx, nt,
               xcd_map);
}

template <int TH>
void launch_sobel_rt(hipStream_t s, const float* in, float* out, int w, int h, uint32_t cap) {
  static int per_cu = 0;
  const int tx = static_cast<int>(ceil_div(w, 64)), nt = tx * static_cast<int>(ceil_div(h, TH));
  const int grid = resident_tile_grid(reinterpret_cast<const void*>(&k_sobel_rt<TH>), 64 * TH / kRowsPerThread,
                                      nt, &per_cu, cap);
  DAGRT_LAUNCH((k_sobel_rt<TH>), dim3(grid), dim3(64 * TH / kRowsPerThread), 0, s, in, out, w, h, tx, nt);
}

hipError_t l_sobel(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const auto* q = static_cast<const dag_p_img*>(p);
  const auto* in = static_cast<const float*>(a[0]);
  auto* out = static_cast<float*>(a[1]);
  const int w = static_cast<int>(q->w), h = static_cast<int>(q->h), xm = static_cast<int>(c.variant & 1);
  if (c.variant == 9) {
    launch_sobel_rt<16>(s, in, out, w, h, c.grid_cap);
    return hipGetLastError();
  }
  if (c.variant == 11) {
    launch_sobel_rt<8>(s, in, out, w, h, c.grid_cap);
    return hipGetLastError();
  }
  switch (c.variant >> 1) {
    case 1: launch_sobel_shape<64, 8>(s, in, out, w, h, xm); break;
    case 2: launch_sobel_shape<64, 4>(s, in, out, w, h, xm); break;
    case 3: launch_sobel_shape<32, 8>(s, in, out, w, h, xm); break;
    default: launch_sobel_shape<64, 16>(s, in, out, w, h, xm); break;
  }
  return hipGetLastError();
}

const char* v_minmax(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t sb) {
  const uint64_t n = pn(p);
  if (n == 0) return "minmax of an empty array";
  if (!mul_fits(n, 4, sz[0])) return "input smaller than 4*n bytes";
  if (sz[1] < 8) return "M smaller than 8 bytes";
  if (reduction_capacity(sb) < 1) return "scratch too small";
  return nullptr;
}
hipError_t l_minmax(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t sb) {
  const uint64_t n = pn(p);
  const int vec = aligned16(a[0]);
  auto* counter = static_cast<uint32_t*>(scr);
  auto* partials = reinterpret_cast<uint64_t*>(static_cast<char*>(scr) + kScratchPartialsOffset);
  const uint32_t g = reduction_grid(vec ? ceil_div(n, 4) : n, c, sb);
  if (c.variant == 1) {
    DAGRT_LAUNCH(k_minmax<true>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                       static_cast<float*>(a[1]), n, vec, counter, partials);
    return hipGetLastError();
  }
  DAGRT_LAUNCH(k_minmax<false>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                     static_cast<float*>(a[1]), n, vec, counter, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DAGRT_LAUNCH(k_finish_minmax, dim3(1), dim3(256), 0, s, partials, g, static_cast<float*>(a[1]));
  return hipGetLastError();
}

const char* v_normalise(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const uint64_t n = pn(p);
  if (!mul_fits(n, 4, sz[0]) || !mul_fits(n, 4, sz[2])) return "S or N smaller than 4*n bytes";
  if (sz[1] < 8) return "M smaller than 8 bytes";
  return nullptr;
}
hipError_t l_normalise(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const uint64_t n = pn(p);
  if (n == 0) return hipSuccess;
  const int vec = aligned16(a[0]) && aligned16(a[2]);
  DAGRT_LAUNCH(k_normalise, dim3(stream_grid(vec ? ceil_div(n, 4) : n, c)), dim3(c.block), 0, s,
                     static_cast<const float*>(a[0]), static_cast<const float*>(a[1]),
                     static_cast<float*>(a[2]), n, vec);
  return hipGetLastError();
}

const char* v_combine(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const uint64_t n = pn(p);
  for (int i = 0; i < 8; ++i)
    if (!mul_fits(n, 4, sz[i])) return "a buffer is smaller than 4*n bytes";
  return nullptr;
}
hipError_t l_combine(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const uint64_t n = pn(p);
  if (n == 0) return hipSuccess;
  int vec = 1;
  for (int i = 0; i < 8; ++i) vec &= aligned16(a[i]) ? 1 : 0;
  DAGRT_LAUNCH(k_unsharp_combine, dim3(stream_grid(vec ? ceil_div(n, 4) : n, c)), dim3(c.block), 0, s,
                     static_cast<const float*>(a[0]), static_cast<const float*>(a[1]),
                     static_cast<const float*>(a[2]), static_cast<const float*>(a[3]),
                     static_cast<const float*>(a[4]), static_cast<const float*>(a[5]),
                     static_cast<const float*>(a[6]), static_cast<float*>(a[7]), n, vec);
  return hipGetLastError();
}

// -- HITS -------------------------------------------------------------------
// Variants 4..16: merge-path tiles of 256 * variant rows and nonzeros;
// 0x100 | IPT: row windows of 256 * IPT nonzeros (at least one tile, which
// owns every row when there is no nonzero).
bool spmv_is_window(uint32_t variant) { return (variant & 0x100u) != 0; }
uint64_t spmv_tiles(const dag_p_csr* q, uint32_t variant) {
  const uint64_t items = 256ull * (variant & 0xffu);
  if (spmv_is_window(variant)) return std::max<uint64_t>(1, ceil_div(static_cast<uint64_t>(q->nnz), items));
  return ceil_div(static_cast<uint64_t>(q->nrows) + q->nnz, items);
}
// Carries live after the reduction ticket counter (which must stay zero):
// head_val, tail_val (fp64), head_row, tail_row, coord (int32, tiles + 1).
// The row-window form uses the first three and keeps its row boundaries
// where coord is.
size_t spmv_scratch_need(uint64_t tiles) { return kScratchPartialsOffset + tiles * (8 + 8 + 4 + 4) + 4 * (tiles + 1); }

const char* v_spmv(const void* p, const size_t* sz, uint32_t, const LaunchCfg& c, size_t sb) {
  const auto* q = static_cast<const dag_p_csr*>(p);
  if (q->nrows == 0) return nullptr;
  if (q->ncols == 0) return "ncols must be > 0";
  if (q->nnz > 0x7fffffffull - q->nrows) return "nrows + nnz must stay below 2^31";
  if (!mul_fits(static_cast<uint64_t>(q->nrows) + 1, 4, sz[0])) return "row_ptr smaller than 4*(nrows+1) bytes";
  if (!mul_fits(q->nnz, 4, sz[1]) || !mul_fits(q->nnz, 4, sz[2])) return "col or val smaller than 4*nnz bytes";
  if (!mul_fits(q->ncols, 4, sz[3])) return "x smaller than 4*ncols bytes";
  if (!mul_fits(q->nrows, 4, sz[4])) return "y smaller than 4*nrows bytes";
  if (spmv_scratch_need(spmv_tiles(q, c.variant)) > sb) return "matrix too large for the per-stream scratch";
  return nullptr;
}

template <int IPT>
void launch_spmv_ipt(hipStream_t s, void* const* a, const dag_p_csr* q, const SpmvScratch& sc, int tiles) {
  DAGRT_LAUNCH(k_spmv_merge<IPT>, dim3(tiles), dim3(256), 0, s, static_cast<const int*>(a[0]),
                     static_cast<const int*>(a[1]), static_cast<const float*>(a[2]),
                     static_cast<const float*>(a[3]), static_cast<float*>(a[4]), static_cast<int>(q->nrows),
                     static_cast<int>(q->ncols), static_cast<int>(q->nnz), sc);
}

SpmvScratch spmv_carries(void* scr, int tiles) {
  char* base = static_cast<char*>(scr) + kScratchPartialsOffset;
  SpmvScratch sc;
  sc.head_val = reinterpret_cast<double*>(base);
  sc.tail_val = reinterpret_cast<double*>(base + 8ull * tiles);
  sc.head_row = reinterpret_cast<int*>(base + 16ull * tiles);
  sc.tail_row = reinterpret_cast<int*>(base + 20ull * tiles);
  sc.coord = reinterpret_cast<int*>(base + 24ull * tiles);
  return sc;
}

hipError_t spmv_partition_into(hipStream_t s, const int* row_ptr, const dag_p_csr* q, uint32_t variant, int tiles,
                               int* coord) {
  const int waves_per_wg = 256 / kWave;
  const int items = static_cast<int>(256 * (variant & 0xffu));
  if (spmv_is_window(variant)) {
    DAGRT_LAUNCH(k_spmv_window_partition, dim3(ceil_div(tiles + 1, waves_per_wg)), dim3(256), 0, s, row_ptr,
                 static_cast<int>(q->nrows), static_cast<int>(q->nnz), items, tiles, coord);
    return hipGetLastError();
  }
  SpmvScratch sc{};
  sc.coord = coord;
  DAGRT_LAUNCH(k_spmv_partition, dim3(ceil_div(tiles + 1, waves_per_wg)), dim3(256), 0, s, row_ptr,
               static_cast<int>(q->nrows), static_cast<int>(q->nnz), items, tiles, sc);
  return hipGetLastError();
}

template <int IPT, bool kStream>
void launch_spmv_window(hipStream_t s, void* const* a, const dag_p_csr* q, const int* own,
                        const SpmvWindowScratch& sc, int tiles) {
  DAGRT_LAUNCH((k_spmv_window<IPT, kStream>), dim3(tiles), dim3(256), 0, s, static_cast<const int*>(a[0]),
               static_cast<const int*>(a[1]), static_cast<const float*>(a[2]), static_cast<const float*>(a[3]),
               static_cast<float*>(a[4]), static_cast<int>(q->nrows), static_cast<int>(q->ncols),
               static_cast<int>(q->nnz), own, sc);
}

// Row-window products and fix-up over the row boundaries in own.
hipError_t spmv_window_fixup(hipStream_t s, void* const* a, const dag_p_csr* q, uint32_t variant, int tiles,
                             const int* own, void* scr, uint32_t cap) {
  const SpmvScratch c = spmv_carries(scr, tiles);
  SpmvWindowScratch sc;
  sc.head_val = c.head_val;
  sc.tail_val = c.tail_val;
  sc.head_row = c.head_row;
  const bool stream = (variant & 0x200u) != 0;
  if (variant & 0x400u) {
    // resident grid: as many workgroups as fit on the GPU at once, never more than the tiles
    // resident workgroups per CU, from the occupancy calculator (once per kernel)
    static int per_cu[2] = {0, 0};
    const int which = (variant & 0xffu) == 8 ? 1 : 0;
    if (per_cu[which] == 0) {
      const void* kf[2] = {reinterpret_cast<const void*>(&k_spmv_window_pf<4>),
                           reinterpret_cast<const void*>(&k_spmv_window_pf<8>)};
      int n = 0;
      const hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kf[which], 256, 0);
      per_cu[which] = (oe == hipSuccess && n > 0) ? n : 4;
    }
    // (grid_cap, if set, leaves the rest of the CUs' slots to kernels on other streams)
    int grid = std::min(tiles, per_cu[which] * device_cus());
    if (cap) grid = std::min<int64_t>(grid, cap);
    grid = std::max(1, grid);
    if ((variant & 0xffu) == 8)
      DAGRT_LAUNCH(k_spmv_window_pf<8>, dim3(grid), dim3(256), 0, s, static_cast<const int*>(a[0]),
                   static_cast<const int*>(a[1]), static_cast<const float*>(a[2]), static_cast<const float*>(a[3]),
                   static_cast<float*>(a[4]), static_cast<int>(q->nrows), static_cast<int>(q->ncols),
                   static_cast<int>(q->nnz), own, tiles, sc);
    else
      DAGRT_LAUNCH(k_spmv_window_pf<4>, dim3(grid), dim3(256), 0, s, static_cast<const int*>(a[0]),
                   static_cast<const int*>(a[1]), static_cast<const float*>(a[2]), static_cast<const float*>(a[3]),
                   static_cast<float*>(a[4]), static_cast<int>(q->nrows), static_cast<int>(q->ncols),
                   static_cast<int>(q->nnz), own, tiles, sc);
  } else
  switch (variant & 0xffu) {
    case 4:
      stream ? launch_spmv_window<4, true>(s, a, q, own, sc, tiles) : launch_spmv_window<4, false>(s, a, q, own, sc, tiles);
      break;
    case 16:
      stream ? launch_spmv_window<16, true>(s, a, q, own, sc, tiles) : launch_spmv_window<16, false>(s, a, q, own, sc, tiles);
      break;
    default:
      stream ? launch_spmv_window<8, true>(s, a, q, own, sc, tiles) : launch_spmv_window<8, false>(s, a, q, own, sc, tiles);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DAGRT_LAUNCH(k_spmv_window_fixup, dim3(ceil_div(tiles, 256)), dim3(256), 0, s, static_cast<const int*>(a[0]),
               static_cast<float*>(a[4]), sc, tiles, static_cast<int>(q->nnz),
               static_cast<int>(256 * (variant & 0xffu)));
  return hipGetLastError();
}

// Merge and fix-up over the tile boundaries in sc.coord.
hipError_t spmv_merge_fixup(hipStream_t s, void* const* a, const dag_p_csr* q, uint32_t ipt, int tiles,
                            const SpmvScratch& sc) {
  switch (ipt) {
    case 4: launch_spmv_ipt<4>(s, a, q, sc, tiles); break;
    case 12: launch_spmv_ipt<12>(s, a, q, sc, tiles); break;
    case 16: launch_spmv_ipt<16>(s, a, q, sc, tiles); break;
    default: launch_spmv_ipt<8>(s, a, q, sc, tiles); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int waves_per_wg = 256 / kWave;
  DAGRT_LAUNCH(k_spmv_fixup, dim3(ceil_div(tiles, waves_per_wg)), dim3(256), 0, s, static_cast<const int*>(a[0]),
               static_cast<float*>(a[4]), sc, tiles, static_cast<int>(q->nnz), static_cast<int>(256 * ipt));
  return hipGetLastError();
}

hipError_t l_spmv(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t) {
  const auto* q = static_cast<const dag_p_csr*>(p);
  if (q->nrows == 0) return hipSuccess;
  const int tiles = static_cast<int>(spmv_tiles(q, c.variant));
  const SpmvScratch sc = spmv_carries(scr, tiles);
  hipError_t e = spmv_partition_into(s, static_cast<const int*>(a[0]), q, c.variant, tiles, sc.coord);
  if (e != hipSuccess) return e;
  if (spmv_is_window(c.variant)) return spmv_window_fixup(s, a, q, c.variant, tiles, sc.coord, scr, c.grid_cap);
  return spmv_merge_fixup(s, a, q, c.variant, tiles, sc);
}

const char* cfg_spmv_rows(const LaunchCfg& c) {
  if (c.block != 256) return "SpMV runs 256-thread workgroups";
  if (c.variant != 4 && c.variant != 8 && c.variant != 16 && c.variant != 32)
    return "spmv_rows variant (lanes per row) must be 4, 8, 16 or 32";
  return nullptr;
}

const char* v_spmv_rows(const void* p, const size_t* sz, uint32_t na, const LaunchCfg& c, size_t sb) {
  const auto* q = static_cast<const dag_p_csr*>(p);
  if (q->nrows == 0) return nullptr;
  if (q->ncols == 0) return "ncols must be > 0";
  if (q->nnz > 0x7fffffffull) return "nnz must stay below 2^31";
  if (!mul_fits(static_cast<uint64_t>(q->nrows) + 1, 4, sz[0])) return "row_ptr smaller than 4*(nrows+1) bytes";
  if (!mul_fits(q->nnz, 4, sz[1]) || !mul_fits(q->nnz, 4, sz[2])) return "col or val smaller than 4*nnz bytes";
  if (!mul_fits(q->ncols, 4, sz[3])) return "x smaller than 4*ncols bytes";
  if (!mul_fits(q->nrows, 4, sz[4])) return "y smaller than 4*nrows bytes";
  return nullptr;
}

template <int L>
void launch_spmv_rows_l(hipStream_t s, void* const* a, const dag_p_csr* q, uint32_t cap) {
  uint64_t g = ceil_div(static_cast<uint64_t>(q->nrows) * L, 256);
  if (cap) g = std::min<uint64_t>(g, cap);
  DAGRT_LAUNCH(k_spmv_rows<L>, dim3(static_cast<uint32_t>(std::max<uint64_t>(g, 1))), dim3(256), 0, s,
                     static_cast<const int*>(a[0]), static_cast<const int*>(a[1]), static_cast<const float*>(a[2]),
                     static_cast<const float*>(a[3]), static_cast<float*>(a[4]), static_cast<int>(q->nrows),
                     static_cast<int>(q->ncols), static_cast<int>(q->nnz));
}

hipError_t l_spmv_rows(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const auto* q = static_cast<const dag_p_csr*>(p);
  if (q->nrows == 0) return hipSuccess;
  switch (c.variant) {
    case 4: launch_spmv_rows_l<4>(s, a, q, c.grid_cap); break;
    case 16: launch_spmv_rows_l<16>(s, a, q, c.grid_cap); break;
    case 32: launch_spmv_rows_l<32>(s, a, q, c.grid_cap); break;
    default: launch_spmv_rows_l<8>(s, a, q, c.grid_cap); break;
  }
  return hipGetLastError();
}

const char* v_sumsq(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t sb) {
  if (!mul_fits(pn(p), 4, sz[0])) return "v smaller than 4*n bytes";
  if (sz[1] < 8) return "s smaller than 8 bytes";
  if (reduction_capacity(sb) < 1) return "scratch too small";
  return nullptr;
}
hipError_t l_sumsq(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t sb) {
  const uint64_t n = pn(p);
  const int vec = aligned16(a[0]);
  auto* counter = static_cast<uint32_t*>(scr);
  auto* partials = reinterpret_cast<uint64_t*>(static_cast<char*>(scr) + kScratchPartialsOffset);
  const uint32_t g = reduction_grid(vec ? ceil_div(n, 4) : n, c, sb);
  if (c.variant == 1) {
    DAGRT_LAUNCH(k_sumsq<true>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                       static_cast<double*>(a[1]), n, vec, counter, partials);
    return hipGetLastError();
  }
  DAGRT_LAUNCH(k_sumsq<false>, dim3(g), dim3(c.block), 0, s, static_cast<const float*>(a[0]),
                     static_cast<double*>(a[1]), n, vec, counter, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DAGRT_LAUNCH(k_finish_sum<double>, dim3(1), dim3(256), 0, s, partials, g, static_cast<double*>(a[1]));
  return hipGetLastError();
}

const char* v_scale(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const uint64_t n = pn(p);
  if (!mul_fits(n, 4, sz[0]) || !mul_fits(n, 4, sz[2])) return "t or v smaller than 4*n bytes";
  if (sz[1] < 8) return "s smaller than 8 bytes";
  return nullptr;
}
hipError_t l_scale(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const uint64_t n = pn(p);
  if (n == 0) return hipSuccess;
  const int vec = aligned16(a[0]) && aligned16(a[2]);
  DAGRT_LAUNCH(k_scale_l2, dim3(stream_grid(vec ? ceil_div(n, 4) : n, c)), dim3(c.block), 0, s,
                     static_cast<const float*>(a[0]), static_cast<const double*>(a[1]),
                     static_cast<float*>(a[2]), n, vec);
  return hipGetLastError();
}

// -- utilities ---------------------------------------------------------------
const char* v_spin(const void* p, const size_t*, uint32_t, const LaunchCfg&, size_t) {
  return static_cast<const dag_p_spin*>(p)->ns <= 1000000000ull ? nullptr : "spin longer than 1 s";
}
hipError_t l_spin(hipStream_t s, void* const*, const void* p, const LaunchCfg&, void*, size_t) {
  const uint64_t ns = static_cast<const dag_p_spin*>(p)->ns;
  const uint64_t ticks = ns * g_wall_khz / 1000000ull;
  DAGRT_LAUNCH(k_spin, dim3(1), dim3(64), 0, s, ticks);
  return hipGetLastError();
}

const char* v_copy(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const uint64_t n = pn(p);
  if (!mul_fits(n, 4, sz[0]) || !mul_fits(n, 4, sz[1])) return "src or dst smaller than 4*n bytes";
  return nullptr;
}
hipError_t l_copy(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const uint64_t n = pn(p);
  if (n == 0) return hipSuccess;
  const int vec = aligned16(a[0]) && aligned16(a[1]);
  DAGRT_LAUNCH(k_copy_f32, dim3(stream_grid(vec ? ceil_div(n, 4) : n, c)), dim3(c.block), 0, s,
                     static_cast<const float*>(a[0]), static_cast<float*>(a[1]), n, vec);
  return hipGetLastError();
}

// -- ML ensemble -------------------------------------------------------------
#define DAGRT_ML_CLASSES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

const dag_p_ml* pml(const void* p) { return static_cast<const dag_p_ml*>(p); }

const char* ml_common(const dag_p_ml* q) {
  if (q->classes < 1 || q->classes > static_cast<uint32_t>(kMlMaxClasses)) return "classes must be in 1..16";
  if (q->features < 1) return "features must be >= 1";
  if (q->reserved) return "reserved must be 0";
  return nullptr;
}

const char* cfg_ridge(const LaunchCfg& c) {
  if (c.variant != 0 && c.variant != 2 && c.variant != 4) return "variant: rows per thread, 0 = one, 2 = two, 4 = four";
  const uint32_t top = c.variant != 0 ? 256 : 512;
  if (c.block < 64 || c.block > top || c.block % 64)
    return "block must be a multiple of 64 in [64, 512] ([64, 256] for variant 4)";
  return nullptr;
}
const char* cfg_ml_one(const LaunchCfg& c) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be a multiple of 64 in [64, 1024]";
  if (c.variant != 0) return "variant must be 0";
  return nullptr;
}

const char* v_nb(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const dag_p_ml* q = pml(p);
  if (const char* e = ml_common(q)) return e;
  if (q->categories < 1) return "categories must be >= 1";
  const uint64_t cfv = static_cast<uint64_t>(q->classes) * q->features * q->categories;
  if (cfv > kNbTable) return "classes * features * categories must be <= 32768 (the LDS table)";
  if (!mul_fits(q->n, 4ull * q->features, sz[0])) return "X smaller than 4*features*n bytes";
  if (sz[1] < 4 * cfv) return "log_theta smaller than 4*classes*features*categories bytes";
  if (sz[2] < 4ull * q->classes) return "log_prior smaller than 4*classes bytes";
  if (!mul_fits(q->n, 4ull * q->classes, sz[3])) return "P smaller than 4*n*classes bytes";
  return nullptr;
}
hipError_t l_nb(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const dag_p_ml* q = pml(p);
  if (q->n == 0) return hipSuccess;
  const dim3 g(stream_grid(q->n, c)), b(c.block);
  const auto* X = static_cast<const float*>(a[0]);
  const auto* lt = static_cast<const float*>(a[1]);
  const auto* lp = static_cast<const float*>(a[2]);
  auto* P = static_cast<float*>(a[3]);
  switch (q->classes) {
#define DAGRT_NB_CASE(K) \
  case K: DAGRT_LAUNCH(k_nb_proba<K>, g, b, 0, s, X, lt, lp, P, q->n, q->features, q->categories); break;
    DAGRT_ML_CLASSES(DAGRT_NB_CASE)
#undef DAGRT_NB_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

uint64_t ridge_lds_bytes(const dag_p_ml* q) { return 8ull * q->features * (q->classes + 1ull); }

const char* v_ridge(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const dag_p_ml* q = pml(p);
  if (const char* e = ml_common(q)) return e;
  if (ridge_lds_bytes(q) > kRidgeLdsBytes) return "features * (classes + 1) must be <= 8192 (the LDS weights)";
  const uint64_t F = q->features, C = q->classes;
  if (!mul_fits(q->n, 4 * F, sz[0])) return "X smaller than 4*n*features bytes";
  if (sz[1] < 4 * F || sz[2] < 4 * F) return "mean or scale smaller than 4*features bytes";
  if (sz[3] < 4 * F * C) return "W smaller than 4*classes*features bytes";
  if (sz[4] < 4 * C) return "b smaller than 4*classes bytes";
  if (!mul_fits(q->n, 4 * C, sz[5])) return "P smaller than 4*n*classes bytes";
  return nullptr;
}
hipError_t l_ridge(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const dag_p_ml* q = pml(p);
  if (q->n == 0) return hipSuccess;
  // four rows per thread need 16-byte aligned float4 columns (n % 4 == 0), else one row
  const bool four = c.variant == 4 && q->n % 4 == 0 && aligned16(a[0]);
  const bool two = c.variant == 2 && q->n % 2 == 0 && reinterpret_cast<uintptr_t>(a[0]) % 8 == 0;
  const dim3 g(stream_grid(four ? q->n / 4 : (two ? q->n / 2 : q->n), c)), b(c.block);
  const size_t shm = ridge_lds_bytes(q);
  const auto* X = static_cast<const float*>(a[0]);
  const auto* mean = static_cast<const float*>(a[1]);
  const auto* scale = static_cast<const float*>(a[2]);
  const auto* W = static_cast<const float*>(a[3]);
  const auto* bias = static_cast<const float*>(a[4]);
  auto* P = static_cast<float*>(a[5]);
  switch (q->classes) {
#define DAGRT_RIDGE_CASE(K)                                                                                \
  case K:                                                                                                  \
    if (four)                                                                                              \
      DAGRT_LAUNCH((k_ridge_proba4<K>), g, b, shm, s, X, mean, scale, W, bias, P, q->n, q->features);      \
    else if (two)                                                                                          \
      DAGRT_LAUNCH((k_ridge_proba2<K>), g, b, shm, s, X, mean, scale, W, bias, P, q->n, q->features);      \
    else                                                                                                   \
      DAGRT_LAUNCH((k_ridge_proba<K>), g, b, shm, s, X, mean, scale, W, bias, P, q->n, q->features);       \
    break;
    DAGRT_ML_CLASSES(DAGRT_RIDGE_CASE)
#undef DAGRT_RIDGE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

const char* v_ensemble(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const dag_p_ml* q = pml(p);
  if (const char* e = ml_common(q)) return e;
  const uint64_t C = q->classes;
  if (!mul_fits(q->n, 4 * C, sz[0]) || !mul_fits(q->n, 4 * C, sz[1]) || !mul_fits(q->n, 4 * C, sz[2]))
    return "Pnb, Prr or avg smaller than 4*n*classes bytes";
  if (!mul_fits(q->n, 4, sz[3])) return "label smaller than 4*n bytes";
  return nullptr;
}
hipError_t l_ensemble(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void*, size_t) {
  const dag_p_ml* q = pml(p);
  if (q->n == 0) return hipSuccess;
  const dim3 g(stream_grid(q->n, c)), b(c.block);
  const auto* pa = static_cast<const float*>(a[0]);
  const auto* pb = static_cast<const float*>(a[1]);
  auto* avg = static_cast<float*>(a[2]);
  auto* label = static_cast<int*>(a[3]);
  switch (q->classes) {
#define DAGRT_ENS_CASE(K) \
  case K: DAGRT_LAUNCH(k_ensemble<K>, g, b, 0, s, pa, pb, avg, label, q->n); break;
    DAGRT_ML_CLASSES(DAGRT_ENS_CASE)
#undef DAGRT_ENS_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// -- DL ---------------------------------------------------------------------------
const char* cfg_conv(const LaunchCfg& c) {
  if (c.block != 256) return "this kernel runs 256-thread workgroups (16 x 16 pooled outputs)";
  if (c.grid_cap != 0) return "grid_cap must be 0";
  if (c.variant > 4)
    return "variant must be 0 (one channel at a time), 1 (channels pipelined), 2 (pipelined, scalar weights), "
           "3 (fp64 matrix cores) or 4 (matrix cores, 16 output channels per workgroup)";
  return nullptr;
}
const dag_p_conv* pconv(const void* p) { return static_cast<const dag_p_conv*>(p); }
uint32_t conv_oc(uint32_t cout) { return cout % 8 == 0 ? 8 : (cout % 4 == 0 ? 4 : 1); }

const char* v_conv(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const dag_p_conv* q = pconv(p);
  if (q->cin < 1 || q->cin > 4096 || q->cout < 1 || q->cout > 4096) return "cin and cout must be in 1..4096";
  if (q->h < 2 || q->w < 2 || q->h % 2 || q->w % 2 || q->h > 65536 || q->w > 65536)
    return "h and w must be even, in 2..65536";
  const uint64_t hw = static_cast<uint64_t>(q->h) * q->w;
  if (sz[0] < 4 * q->cin * hw) return "x smaller than 4*cin*h*w bytes";
  if (sz[1] < 36ull * q->cout * q->cin) return "w smaller than 4*cout*cin*9 bytes";
  if (sz[2] < 4ull * q->cout) return "b smaller than 4*cout bytes";
  if (sz[3] < 4 * q->cout * (hw / 4)) return "y smaller than 4*cout*(h/2)*(w/2) bytes";
  const uint64_t tiles = ceil_div(q->h / 2, kConvTile) * ceil_div(q->w / 2, kConvTile);
  if (tiles > (1u << 30) || q->cout / conv_oc(q->cout) > 65535) return "grid too large";
  const uint64_t mtiles = ceil_div(q->h, kConvMfmaTile) * ceil_div(q->w, kConvMfmaTile);
  if (mtiles > (1u << 30)) return "grid too large";
  return nullptr;
}
hipError_t l_conv(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t sb) {
  const dag_p_conv* q = pconv(p);
  const uint32_t tiles_x = static_cast<uint32_t>(ceil_div(q->w / 2, kConvTile));
  const uint32_t tiles_y = static_cast<uint32_t>(ceil_div(q->h / 2, kConvTile));
  const uint32_t oc = conv_oc(q->cout);
  const dim3 g(tiles_x * tiles_y, q->cout / oc), b(c.block);
  const auto* x = static_cast<const float*>(a[0]);
  const auto* w = static_cast<const float*>(a[1]);
  const auto* bias = static_cast<const float*>(a[2]);
  auto* y = static_cast<float*>(a[3]);
  // variants 3 and 4: the matrix-core form where the channel counts allow it
  // (conv_mfma_njb; 4 with one block of 16 output channels per workgroup),
  // else variant 1
  uint32_t njb = c.variant >= 3 ? conv_mfma_njb(q->cin, q->cout) : 0;
  if (c.variant == 4 && njb == 2) njb = 1;  // 16 output channels per workgroup: twice the workgroups
  if (njb) {
    const uint32_t mtx = static_cast<uint32_t>(ceil_div(q->w, kConvMfmaTile));
    const uint32_t mty = static_cast<uint32_t>(ceil_div(q->h, kConvMfmaTile));
    const size_t lds = conv_mfma_lds(q->cin, njb);
    const dim3 mg(mtx * mty, q->cout / (16 * njb));
    if (njb == 2)
      DAGRT_LAUNCH(k_conv3x3_relu_pool_mfma<2>, mg, dim3(256), lds, s, x, w, bias, y, q->cin, q->h, q->w, mtx);
    else
      DAGRT_LAUNCH(k_conv3x3_relu_pool_mfma<1>, mg, dim3(256), lds, s, x, w, bias, y, q->cin, q->h, q->w, mtx);
    return hipGetLastError();
  }
  // variant 2 needs the fp64 weight copy in the stream's scratch (above the
  // counters); where it does not fit, variant 1 runs instead
  const uint64_t nw = static_cast<uint64_t>(q->cin) * q->cout * 9;
  const bool sw = c.variant == 2 && nw <= reduction_capacity(sb);
  double* w64 = sw ? reinterpret_cast<double*>(static_cast<char*>(scr) + kScratchPartialsOffset) : nullptr;
  if (sw) {
    const uint32_t gw = static_cast<uint32_t>(std::min<uint64_t>(ceil_div(nw, 256), 1024));
    DAGRT_LAUNCH(k_conv_weights_f64, dim3(gw), dim3(256), 0, s, w, w64, q->cin, q->cout);
  }
  if (c.variant != 0) {  // 1, 2, and 3 where the matrix-core form does not apply
#define DAGRT_CONV_PIPE(OC)                                                                                  \
  if (sw)                                                                                                    \
    DAGRT_LAUNCH((k_conv3x3_relu_pool_pipe<OC, true>), g, b, 0, s, x, w, w64, bias, y, q->cin, q->cout, q->h, \
                 q->w, tiles_x);                                                                             \
  else                                                                                                       \
    DAGRT_LAUNCH((k_conv3x3_relu_pool_pipe<OC, false>), g, b, 0, s, x, w, w64, bias, y, q->cin, q->cout,     \
                 q->h, q->w, tiles_x);
    if (oc == 8) {
      DAGRT_CONV_PIPE(8)
    } else if (oc == 4) {
      DAGRT_CONV_PIPE(4)
    } else {
      DAGRT_CONV_PIPE(1)
    }
#undef DAGRT_CONV_PIPE
  } else if (oc == 8) {
    DAGRT_LAUNCH(k_conv3x3_relu_pool<8>, g, b, 0, s, x, w, bias, y, q->cin, q->h, q->w, tiles_x);
  } else if (oc == 4) {
    DAGRT_LAUNCH(k_conv3x3_relu_pool<4>, g, b, 0, s, x, w, bias, y, q->cin, q->h, q->w, tiles_x);
  } else {
    DAGRT_LAUNCH(k_conv3x3_relu_pool<1>, g, b, 0, s, x, w, bias, y, q->cin, q->h, q->w, tiles_x);
  }
  return hipGetLastError();
}

const char* cfg_dense(const LaunchCfg& c) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be a multiple of 64 in [64, 1024]";
  if (c.variant > 4)
    return "variant must be 0 (one input per lane), 1 or 2 (contiguous 1 KB loads, 2 or 4 chunks in flight), "
           "3 or 4 (the same with the final add in a second kernel)";
  return nullptr;
}
const dag_p_dense* pdense(const void* p) { return static_cast<const dag_p_dense*>(p); }
uint32_t dense_grid(const dag_p_dense* q, const LaunchCfg& c, size_t sb) {
  uint64_t g = stream_grid(q->n, c);
  g = std::min<uint64_t>(g, reduction_capacity(sb) / kDenseMaxOut);
  return static_cast<uint32_t>(std::max<uint64_t>(g, 1));
}
const char* v_dense(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t sb) {
  const dag_p_dense* q = pdense(p);
  if (q->m < 1 || q->m > static_cast<uint32_t>(kDenseMaxOut)) return "m must be in 1..16";
  if (q->reserved) return "reserved must be 0";
  if (!mul_fits(q->n, 4, sz[0])) return "x smaller than 4*n bytes";
  if (!mul_fits(q->n, 4ull * q->m, sz[1])) return "W smaller than 4*n*m bytes";
  if (sz[2] < 4ull * q->m || sz[3] < 4ull * q->m) return "b or y smaller than 4*m bytes";
  if (reduction_capacity(sb) < static_cast<uint64_t>(kDenseMaxOut)) return "scratch too small";
  return nullptr;
}
hipError_t l_dense(hipStream_t s, void* const* a, const void* p, const LaunchCfg& c, void* scr, size_t sb) {
  const dag_p_dense* q = pdense(p);
  auto* counter = static_cast<uint32_t*>(scr);
  auto* partials = reinterpret_cast<uint64_t*>(static_cast<char*>(scr) + kScratchPartialsOffset);
  const int vec = aligned16(a[1]);
  const dim3 g(dense_grid(q, c, sb)), b(c.block);
  const auto* x = static_cast<const float*>(a[0]);
  const auto* W = static_cast<const float*>(a[1]);
  const auto* bias = static_cast<const float*>(a[2]);
  auto* y = static_cast<float*>(a[3]);
  // variants 1 to 4 where their load pattern applies (M of 4, 8 or 16, aligned W):
  // 1, 2: 2 or 4 chunks in flight, last block adds; 3, 4: the same, final add
  // in a second kernel
  if (c.variant != 0 && vec && (q->m == 4 || q->m == 8 || q->m == 16)) {
#define DAGRT_DENSE_LANES(U, SPLIT)                                                                     \
  if (q->m == 4)                                                                                        \
    DAGRT_LAUNCH((k_dense_lanes<4, U, SPLIT>), g, b, 0, s, x, W, bias, y, q->n, counter, partials);     \
  else if (q->m == 8)                                                                                   \
    DAGRT_LAUNCH((k_dense_lanes<8, U, SPLIT>), g, b, 0, s, x, W, bias, y, q->n, counter, partials);     \
  else                                                                                                  \
    DAGRT_LAUNCH((k_dense_lanes<16, U, SPLIT>), g, b, 0, s, x, W, bias, y, q->n, counter, partials);
    const bool split = c.variant >= 3;
    if (c.variant == 1) {
      DAGRT_DENSE_LANES(2, false)
    } else if (c.variant == 2) {
      DAGRT_DENSE_LANES(4, false)
    } else if (c.variant == 3) {
      DAGRT_DENSE_LANES(2, true)
    } else {
      DAGRT_DENSE_LANES(4, true)
    }
#undef DAGRT_DENSE_LANES
    if (split) {
      const uint32_t nb = g.x;
      if (q->m == 4)
        DAGRT_LAUNCH(k_dense_final<4>, dim3(1), dim3(1024), 0, s, partials, nb, bias, y);
      else if (q->m == 8)
        DAGRT_LAUNCH(k_dense_final<8>, dim3(1), dim3(1024), 0, s, partials, nb, bias, y);
      else
        DAGRT_LAUNCH(k_dense_final<16>, dim3(1), dim3(1024), 0, s, partials, nb, bias, y);
    }
    return hipGetLastError();
  }
  switch (q->m) {
#define DAGRT_DENSE_CASE(K) \
  case K: DAGRT_LAUNCH(k_dense<K>, g, b, 0, s, x, W, bias, y, q->n, vec, counter, partials); break;
    DAGRT_ML_CLASSES(DAGRT_DENSE_CASE)
#undef DAGRT_DENSE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

const char* cfg_combine(const LaunchCfg& c) {
  if (c.block != 64 || c.grid_cap != 0 || c.variant != 0) return "this kernel runs one 64-thread workgroup";
  return nullptr;
}
const char* v_combine2(const void* p, const size_t* sz, uint32_t, const LaunchCfg&, size_t) {
  const auto* q = static_cast<const dag_p_combine*>(p);
  if (q->m < 1 || q->m > 32) return "m must be in 1..32";
  if (q->reserved) return "reserved must be 0";
  if (sz[0] < 4ull * q->m || sz[1] < 4ull * q->m) return "e1 or e2 smaller than 4*m bytes";
  if (sz[2] < 8ull * q->m) return "w smaller than 8*m bytes";
  if (sz[3] < 4 || sz[4] < 4) return "b or p smaller than 4 bytes";
  return nullptr;
}
hipError_t l_combine2(hipStream_t s, void* const* a, const void* p, const LaunchCfg&, void*, size_t) {
  const auto* q = static_cast<const dag_p_combine*>(p);
  DAGRT_LAUNCH(k_siamese_combine, dim3(1), dim3(64), 0, s, static_cast<const float*>(a[0]),
               static_cast<const float*>(a[1]), static_cast<const float*>(a[2]), static_cast<const float*>(a[3]),
               static_cast<float*>(a[4]), q->m);
  return hipGetLastError();
}

const KernelDesc kTable[] = {
    /* 0 */ {nullptr, 0, 0, 0, {0, 0, 0}, nullptr, nullptr, nullptr},
    /* 1 */ {"vec_square", 1, 0x1, sizeof(dag_p_n), {256, 0, 0}, v_vec_square, l_vec_square, cfg_block_any},
    /* 2 */ {"vec_sum_diff", 3, 0x4, sizeof(dag_p_n), {256, 1024, 0}, v_vec_sum_diff, l_vec_sum_diff, cfg_reduce},
    /* 3 */ {"bs_call", 2, 0x2, sizeof(dag_p_bs), {256, 0, 0}, v_bs, l_bs, cfg_bs},
    /* 4 */ {"gauss_blur", 2, 0x2, sizeof(dag_p_img), {256, 0, 1}, v_blur, l_blur, cfg_tile},
    /* 5 */ {"sobel", 2, 0x2, sizeof(dag_p_img), {256, 0, 1}, v_img2, l_sobel, cfg_tile},
    /* 6 */ {"minmax", 2, 0x2, sizeof(dag_p_n), {256, 1024, 0}, v_minmax, l_minmax, cfg_reduce},
    /* 7 */ {"normalise", 3, 0x4, sizeof(dag_p_n), {256, 0, 0}, v_normalise, l_normalise, cfg_block_any},
    /* 8 */ {"unsharp_combine", 8, 0x80, sizeof(dag_p_n), {256, 0, 0}, v_combine, l_combine, cfg_block_any},
    /* 9 */ {"spmv", 5, 0x10, sizeof(dag_p_csr), {256, 0, 8}, v_spmv, l_spmv, cfg_spmv},
    /* 10 */ {"spmv_rows", 5, 0x10, sizeof(dag_p_csr), {256, 0, 8}, v_spmv_rows, l_spmv_rows, cfg_spmv_rows},
    /* 11 */ {"sumsq", 2, 0x2, sizeof(dag_p_n), {256, 1024, 0}, v_sumsq, l_sumsq, cfg_reduce},
    /* 12 */ {"scale_l2", 3, 0x4, sizeof(dag_p_n), {256, 0, 0}, v_scale, l_scale, cfg_block_any},
    /* 13 */ {"spin", 0, 0x0, sizeof(dag_p_spin), {64, 0, 0}, v_spin, l_spin, cfg_spin},
    /* 14 */ {"copy_f32", 2, 0x2, sizeof(dag_p_n), {256, 0, 0}, v_copy, l_copy, cfg_block_any},
    /* 15 */ {"nb_proba", 4, 0x8, sizeof(dag_p_ml), {1024, 256, 0}, v_nb, l_nb, cfg_ml_one},
    /* 16 */ {"ridge_proba", 6, 0x20, sizeof(dag_p_ml), {256, 0, 0}, v_ridge, l_ridge, cfg_ridge},
    /* 17 */ {"ensemble", 4, 0xC, sizeof(dag_p_ml), {256, 0, 0}, v_ensemble, l_ensemble, cfg_ml_one},
    /* 18 */ {"conv3x3_relu_pool", 4, 0x8, sizeof(dag_p_conv), {256, 0, 1}, v_conv, l_conv, cfg_conv},
    /* 19 */ {"dense", 4, 0x8, sizeof(dag_p_dense), {512, 512, 4}, v_dense, l_dense, cfg_dense},
    /* 20 */ {"siamese_combine", 5, 0x10, sizeof(dag_p_combine), {64, 0, 0}, v_combine2, l_combine2, cfg_combine},
};

static_assert(sizeof(kTable) / sizeof(kTable[0]) == kNumBuiltin, "kernel table and kNumBuiltin disagree");

}  // namespace

const KernelDesc* builtin_kernel(uint32_t id) {
  if (id >= sizeof(kTable) / sizeof(kTable[0])) return nullptr;
  return kTable[id].name ? &kTable[id] : nullptr;
}

uint64_t spmv_plan_ints(const void* params, const LaunchCfg& cfg) {
  const auto* q = static_cast<const dag_p_csr*>(params);
  return q->nrows == 0 ? 0 : spmv_tiles(q, cfg.variant) + 1;
}

hipError_t spmv_plan(hipStream_t s, const int* row_ptr, const void* params, const LaunchCfg& cfg, int* coord) {
  const auto* q = static_cast<const dag_p_csr*>(params);
  if (q->nrows == 0) return hipSuccess;
  return spmv_partition_into(s, row_ptr, q, cfg.variant, static_cast<int>(spmv_tiles(q, cfg.variant)), coord);
}

hipError_t spmv_planned(hipStream_t s, void* const* ptrs, const void* params, const LaunchCfg& cfg,
                        const int* coord, void* scratch) {
  const auto* q = static_cast<const dag_p_csr*>(params);
  if (q->nrows == 0) return hipSuccess;
  const int tiles = static_cast<int>(spmv_tiles(q, cfg.variant));
  if (spmv_is_window(cfg.variant))
    return spmv_window_fixup(s, ptrs, q, cfg.variant, tiles, coord, scratch, cfg.grid_cap);
  SpmvScratch sc = spmv_carries(scratch, tiles);
  sc.coord = const_cast<int*>(coord);
  return spmv_merge_fixup(s, ptrs, q, cfg.variant, tiles, sc);
}

hipError_t copy_by_kernel(hipStream_t s, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  constexpr uint32_t kCopyWorkgroups = 128;  // enough requests in flight to fill the link
  hipLaunchKernelGGL(k_copy_bytes, dim3(kCopyWorkgroups), dim3(256), 0, s, static_cast<const uint8_t*>(src),
                     static_cast<uint8_t*>(dst), static_cast<uint64_t>(bytes));
  return hipGetLastError();
}

hipError_t release_l2(hipStream_t s) {
  constexpr uint32_t kReleaseWorkgroups = 64;
  hipLaunchKernelGGL(k_release_l2, dim3(kReleaseWorkgroups), dim3(64), 0, s);
  return hipGetLastError();
}

hipError_t signal_raise(hipStream_t s, uint64_t* word, uint64_t value) {
  hipLaunchKernelGGL(k_dag_signal, dim3(1), dim3(64), 0, s, word, value);
  return hipGetLastError();
}

hipError_t signal_wait(hipStream_t s, const SignalWaits& w) {
  if (w.n == 0) return hipSuccess;
  if (w.n > kMaxSignalWaits) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dag_wait, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

uint64_t wall_clock_ticks_per_ms() { return g_wall_khz; }

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  tl_start = start;
  tl_stop = stop;
}

void set_wall_clock_khz(uint64_t khz) {
  if (khz) g_wall_khz = khz;
}

}  // namespace dagrt
