// Pass 2 of the estimator: theta~_i = || A[i, K] Z ||^2 (Algorithm 8, last
// step, on the selected columns; the row-norm computation the paper singles
// out as the floor of every algorithm of its framework, Section 2.1).
//
// Z_full (d x k) holds Z's rows at the selected columns' ids and zeros
// elsewhere, so A[i, K] Z = A[i, :] Z_full and A is read in its natural
// layout with no gather.  Each wave owns 16-row tiles; per tile it streams
// the 16 rows straight from HBM into registers (16-byte loads, 64 bytes of
// each row per instruction) and feeds them as the A operand of the matrix
// cores, with Z_full as the B operand.  Because the contraction index may be
// permuted freely as long as A and Z use the same permutation, each lane's
// 16-byte vector is used as-is: for chunk t, lane group g = l/16 covers
// columns t*CW + EL*g + (0..EL-1), and Z_full is packed in that order
// (trsm.hip).  The 16 x k product never leaves the accumulators: squares
// are summed per lane and across the 16 lanes of a row with shuffles.
//
// Variants (LEV_AZ_*): FP64 (16x16x4f64, EL 2), FP32 (16x16x4f32, EL 4; A
// may be stored as FP32 or BF16) and BF16x3 for FP32 A (BF16 storage with Z
// in one, two or three BF16 parts runs in rownorm_bf16.hip):
// A and Z are each split exactly into three BF16 parts (hi + mid + lo, 24
// significant bits, like FP32) and the six products above 2^-24 relative
// (hh, hm, mh, hl, mm, lh) run on the BF16 matrix cores, which on gfx950
// deliver 16x the FP32 matrix rate: the FP32-accurate pass becomes bound by
// HBM instead of by FP32 MFMA throughput.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lev_internal.h"

namespace lev {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---- per-variant traits ----------------------------------------------------
template <int VAR, typename TA>
struct Frag;

// FP64: two doubles per lane, 16-byte load.
template <>
struct Frag<0, double> {
  static constexpr int EL = 2, CW = 8, NZ = 1;
  using T = uint4;
  __device__ static T load(const double* row, int64_t col, int64_t d, bool ok) {
    if (!ok || col >= d) return make_uint4(0u, 0u, 0u, 0u);
    uint4 v = *reinterpret_cast<const uint4*>(row + col);
    if (col + 1 >= d) v.z = v.w = 0u;
    return v;
  }
};

// FP32 from FP32 storage: four floats, 16-byte load.
template <>
struct Frag<1, float> {
  static constexpr int EL = 4, CW = 16, NZ = 1;
  using T = uint4;
  __device__ static T load(const float* row, int64_t col, int64_t d, bool ok) {
    if (!ok || col >= d) return make_uint4(0u, 0u, 0u, 0u);
    uint4 v = *reinterpret_cast<const uint4*>(row + col);
    if (col + 3 >= d) {
      if (col + 1 >= d) v.y = 0u;
      if (col + 2 >= d) v.z = 0u;
      v.w = 0u;
    }
    return v;
  }
};

// FP32 from BF16 storage: four bf16 (8-byte load), widened exactly.
template <>
struct Frag<1, __hip_bfloat16> {
  static constexpr int EL = 4, CW = 16, NZ = 1;
  using T = uint4;
  __device__ static T load(const __hip_bfloat16* row, int64_t col, int64_t d, bool ok) {
    if (!ok || col >= d) return make_uint4(0u, 0u, 0u, 0u);
    const uint2 v = *reinterpret_cast<const uint2*>(row + col);
    uint4 o = make_uint4(v.x << 16, v.x & 0xFFFF0000u, v.y << 16, v.y & 0xFFFF0000u);
    if (col + 3 >= d) {
      if (col + 1 >= d) o.y = 0u;
      if (col + 2 >= d) o.z = 0u;
      o.w = 0u;
    }
    return o;
  }
};

// BF16x3 from FP32 storage: eight floats (two 16-byte loads).
struct F8 {
  uint4 lo, hi;
};
template <>
struct Frag<4, float> {
  static constexpr int EL = 8, CW = 32, NZ = 3;
  using T = F8;
  __device__ static T load(const float* row, int64_t col, int64_t d, bool ok) {
    F8 f{make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u)};
    if (!ok || col >= d) return f;
    f.lo = *reinterpret_cast<const uint4*>(row + col);
    if (col + 4 < d) f.hi = *reinterpret_cast<const uint4*>(row + col + 4);
    if (col + 7 >= d) {
      uint32_t w[8] = {f.lo.x, f.lo.y, f.lo.z, f.lo.w, f.hi.x, f.hi.y, f.hi.z, f.hi.w};
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (col + e >= d) w[e] = 0u;
      f.lo = make_uint4(w[0], w[1], w[2], w[3]);
      f.hi = make_uint4(w[4], w[5], w[6], w[7]);
    }
    return f;
  }
};

template <int VAR>
struct Acc {
  using T = v4f;
};
template <>
struct Acc<0> {
  using T = v4d;
};

typedef float v8f __attribute__((ext_vector_type(8)));

// x = h + m + l exactly (for normal numbers): each part is the
// round-to-nearest BF16 of what the previous parts left over.
__device__ __forceinline__ void split3(const F8& f, v8bf& h, v8bf& m, v8bf& l) {
  const v8f x = {__uint_as_float(f.lo.x), __uint_as_float(f.lo.y), __uint_as_float(f.lo.z),
                 __uint_as_float(f.lo.w), __uint_as_float(f.hi.x), __uint_as_float(f.hi.y),
                 __uint_as_float(f.hi.z), __uint_as_float(f.hi.w)};
  h = __builtin_convertvector(x, v8bf);
  const v8f r1 = x - __builtin_convertvector(h, v8f);
  m = __builtin_convertvector(r1, v8bf);
  const v8f r2 = r1 - __builtin_convertvector(m, v8f);
  l = __builtin_convertvector(r2, v8bf);
}

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// The same split with one packed conversion per pair of values; the BF16
// parts are widened back to FP32 by shifting them into the high half, which
// is exact, so the parts equal those of split3 bit for bit.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}
__device__ __forceinline__ void split3_pk(const F8& f, v8bf& h, v8bf& m, v8bf& l) {
  const uint32_t w[8] = {f.lo.x, f.lo.y, f.lo.z, f.lo.w, f.hi.x, f.hi.y, f.hi.z, f.hi.w};
  uint32_t hp[4], mp[4], lp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float x0 = __uint_as_float(w[2 * j]), x1 = __uint_as_float(w[2 * j + 1]);
    hp[j] = pk_bf16(x0, x1);
    const float r0 = x0 - __uint_as_float(hp[j] << 16), r1 = x1 - __uint_as_float(hp[j] & 0xFFFF0000u);
    mp[j] = pk_bf16(r0, r1);
    const float s0 = r0 - __uint_as_float(mp[j] << 16), s1 = r1 - __uint_as_float(mp[j] & 0xFFFF0000u);
    lp[j] = pk_bf16(s0, s1);
  }
  h = __builtin_bit_cast(v8bf, make_uint4(hp[0], hp[1], hp[2], hp[3]));
  m = __builtin_bit_cast(v8bf, make_uint4(mp[0], mp[1], mp[2], mp[3]));
  l = __builtin_bit_cast(v8bf, make_uint4(lp[0], lp[1], lp[2], lp[3]));
}

__device__ __forceinline__ v4f mfma_bf16(const v8bf& a, const v8bf& b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v8bf as_bf(const uint4& u) { return __builtin_bit_cast(v8bf, u); }

// acc += A_frag * Z_frag over one chunk of the contraction; z[p] is the
// p-th part of Z's fragment (NZ parts).
template <int VAR, typename TF>
__device__ __forceinline__ void mma(typename Acc<VAR>::T& acc, const TF& a, const uint4* z);

template <>
__device__ __forceinline__ void mma<0, uint4>(v4d& acc, const uint4& a, const uint4* z) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double((int)a.y, (int)a.x),
                                             __hiloint2double((int)z[0].y, (int)z[0].x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double((int)a.w, (int)a.z),
                                             __hiloint2double((int)z[0].w, (int)z[0].z), acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<1, uint4>(v4f& acc, const uint4& a, const uint4* z) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(z[0].x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(z[0].y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(z[0].z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(z[0].w), acc, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T sum16(T x) {
  // reduce over the 16 lanes sharing l / 16 (xor over the low 4 bits)
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

constexpr int kThreads = 512;
// Chunks loaded per batch (loads in flight per lane).  BF16x3 keeps its
// batch at 4 so the kernel stays under 128 VGPRs (four waves per SIMD).
template <int VAR>
constexpr int batch_of() { return VAR == 4 ? 4 : 8; }
// Chunks accumulated in FP32 before the flush into FP64 (one: flushing
// every second chunk saves ~3% of the pass and triples the worst FP32
// error on small coherent inputs).
template <int VAR>
constexpr int flush_of() { return 1; }

// Zpack: part p of vector (t, cb, lane) at index p * part_vecs + (t*CB + cb)*64 + lane.
template <int VAR, typename TA, int CB, bool ZLDS>
__global__ __launch_bounds__(kThreads) void rownorm_dense_kernel(const TA* __restrict__ A, int64_t n,
                                                                 int64_t d, int64_t ld, int64_t nt,
                                                                 const uint4* __restrict__ Zg,
                                                                 int64_t zvecs, int64_t part_vecs,
                                                                 void* __restrict__ theta, ColTile ct) {
  using F = Frag<VAR, TA>;
  using AccT = typename Acc<VAR>::T;
  constexpr int kBatch = batch_of<VAR>();
  extern __shared__ uint4 zs[];
  if (col_tile_dead(ct)) return;
  const uint4* Z = Zg;
  if constexpr (ZLDS) {
    for (int64_t i = threadIdx.x; i < zvecs; i += kThreads) zs[i] = Zg[i];
    __syncthreads();
    Z = zs;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int64_t ntiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * (kThreads / 64) + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * (kThreads / 64)) {
    const int64_t row = tile * 16 + (lane & 15);
    const bool ok = row < n;
    const TA* rp = A + (ok ? row : 0) * ld;
    AccT acc[CB];
    // FP32 forms: the matrix-core accumulator is flushed into FP64 after
    // every flush_of<VAR>() chunks, so FP32 rounding only ever sums a few
    // dozen products.
    double acc64[CB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      acc[cb] = AccT{};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[cb][v] = 0.0;
    }
    for (int64_t t0 = 0; t0 < nt; t0 += kBatch) {
      typename F::T a[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t t = t0 + u;
        a[u] = F::load(rp, t * F::CW + F::EL * g, d, ok && t < nt);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t t = t0 + u;
        if (t < nt) {
          if constexpr (VAR == 4) {
            v8bf ah, am, al;
            split3(a[u], ah, am, al);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int64_t zi = (t * CB + cb) * 64 + lane;
              const v8bf zh = as_bf(Z[zi]), zm = as_bf(Z[zi + part_vecs]), zl = as_bf(Z[zi + 2 * part_vecs]);
              v4f c = acc[cb];
              c = mfma_bf16(al, zh, c);  // smallest terms first
              c = mfma_bf16(am, zm, c);
              c = mfma_bf16(ah, zl, c);
              c = mfma_bf16(am, zh, c);
              c = mfma_bf16(ah, zm, c);
              c = mfma_bf16(ah, zh, c);
              acc[cb] = c;
            }
          } else {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int64_t zi = (t * CB + cb) * 64 + lane;
              uint4 zp[F::NZ];
#pragma unroll
              for (int p = 0; p < F::NZ; ++p) zp[p] = Z[zi + p * part_vecs];
              mma<VAR, typename F::T>(acc[cb], a[u], zp);
            }
          }
          if constexpr (VAR != 0) {
            if ((u + 1) % flush_of<VAR>() == 0 || t + 1 == nt) {
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[cb][v] += (double)acc[cb][v];
                acc[cb] = AccT{};
              }
            }
          }
        }
      }
    }
    if constexpr (VAR == 0) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[cb][v] = acc[cb][v];
    }
    // theta for the rows held by lane group g (rows 4 g + v for the f32
    // accumulators, g + 4 v for f64): sum of squares over the 16 lanes of the
    // group and the CB column tiles.
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) s[v] = fma(acc64[cb][v], acc64[cb][v], s[v]);
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = sum16(s[v]);
    if ((lane & 15) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = tile * 16 + (VAR == 0 ? g + 4 * v : 4 * g + v);
        if (r < n) {
          if constexpr (VAR == 0) {
            double* th = static_cast<double*>(theta);
            th[r] = ct.acc ? th[r] + s[v] : s[v];
          } else {
            float* th = static_cast<float*>(theta);
            th[r] = ct.acc ? th[r] + (float)s[v] : (float)s[v];
          }
        }
      }
    }
  }
}

constexpr size_t kMaxLdsZ = 144 * 1024;

// BF16x3 over FP32 rows with Z staged in LDS (the dense FP32 workload's
// pass).  Two shapes of workgroup: 768 threads when two copies of Z fit in a
// CU's LDS (24 waves per CU, two chunks in flight per wave: more waves with
// fewer registers each keep more of HBM's latency covered than fewer waves
// with deeper batches), else 1024 threads and one workgroup per CU.
//  * Z is staged with every load of a thread in flight before its first LDS
//    store (a load-store loop would pay one L2 round trip per vector).
//  * Tiles whose 16 rows all exist, when d is a multiple of 32, take a path
//    with no per-element checks: one base address per lane, the chunk
//    offsets folded into the load instructions.  The last partial tile and
//    ragged d take the masked path: each load reads an address that holds
//    valid data (its own, else the row start) and invalid parts are zeroed.
//  * Per chunk the six products accumulate from zero in FP32 and are added
//    to the FP64 accumulators, as in rownorm_dense_kernel.
template <int WG>
struct X3Shape;
template <>
struct X3Shape<768> {
  static constexpr int kMinWaves = 6, kBatch = 2, kMaxZVecs = 80 * 1024 / 16;
};
template <>
struct X3Shape<1024> {
  static constexpr int kMinWaves = 4, kBatch = 4, kMaxZVecs = (int)(kMaxLdsZ / 16);
};

template <int CB, int WG>
__global__ __launch_bounds__(WG, X3Shape<WG>::kMinWaves) void rownorm_x3_kernel(
    const float* __restrict__ A, int64_t n, int64_t d, int64_t ld, int64_t nt, const uint4* __restrict__ Zg,
    int64_t zvecs, int64_t part_vecs, void* __restrict__ theta_out, ColTile ct) {
  constexpr int kB = X3Shape<WG>::kBatch;
  constexpr int kZPer = (X3Shape<WG>::kMaxZVecs + WG - 1) / WG;
  constexpr int kWaves = WG / 64;
  if (col_tile_dead(ct)) return;
  float* theta = static_cast<float*>(theta_out);
  const bool theta_vec = (reinterpret_cast<uintptr_t>(theta) & 15) == 0;
  extern __shared__ uint4 zs[];
  {
    // indexes past the end load and store the last vector again (same value)
    uint4 zt[kZPer];
#pragma unroll
    for (int j = 0; j < kZPer; ++j) {
      const int64_t i = threadIdx.x + (int64_t)j * WG;
      zt[j] = Zg[i < zvecs ? i : zvecs - 1];
    }
#pragma unroll
    for (int j = 0; j < kZPer; ++j) {
      const int64_t i = threadIdx.x + (int64_t)j * WG;
      zs[i < zvecs ? i : zvecs - 1] = zt[j];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int64_t ntiles = (n + 15) / 16;
  const bool whole = (d % 32) == 0;
  // the workgroup index runs fastest over the tiles, so when the tile count
  // is not a multiple of the resident waves the last round's tiles are spread
  // over every workgroup (and CU) instead of filling the first few
  for (int64_t tile = (int64_t)wave * gridDim.x + blockIdx.x; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t row = tile * 16 + (lane & 15);
    const bool ok = row < n;
    const float* rp = A + (ok ? row : 0) * ld;
    double acc64[CB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[cb][v] = 0.0;
    auto chunks = [&](auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const float* lp = rp + 8 * g;
      for (int64_t t0 = 0; t0 < nt; t0 += kB) {
        F8 a[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int64_t t = t0 + u;
          if constexpr (FULL) {
            const float* p = lp + (t < nt ? t : 0) * 32;
            a[u].lo = *reinterpret_cast<const uint4*>(p);
            a[u].hi = *reinterpret_cast<const uint4*>(p + 4);
          } else {
            const int64_t col = t * 32 + 8 * g;
            const bool vlo = ok && t < nt && col < d;
            const bool vhi = vlo && col + 4 < d;
            a[u].lo = *reinterpret_cast<const uint4*>(rp + (vlo ? col : 0));
            a[u].hi = *reinterpret_cast<const uint4*>(rp + (vhi ? col + 4 : 0));
          }
        }
        if constexpr (!FULL) {
#pragma unroll
          for (int u = 0; u < kB; ++u) {
            const int64_t t = t0 + u;
            const int64_t col = t * 32 + 8 * g;
            uint32_t w[8] = {a[u].lo.x, a[u].lo.y, a[u].lo.z, a[u].lo.w, a[u].hi.x, a[u].hi.y, a[u].hi.z, a[u].hi.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (!ok || t >= nt || col + e >= d) w[e] = 0u;
            a[u].lo = make_uint4(w[0], w[1], w[2], w[3]);
            a[u].hi = make_uint4(w[4], w[5], w[6], w[7]);
          }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int64_t t = t0 + u;
          if (t < nt) {
            v8bf ah, am, al;
            split3_pk(a[u], ah, am, al);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int zi = ((int)t * CB + cb) * 64 + lane;
              const v8bf zh = as_bf(zs[zi]), zm = as_bf(zs[zi + part_vecs]), zl = as_bf(zs[zi + 2 * part_vecs]);
              v4f c = v4f{};
              c = mfma_bf16(al, zh, c);  // smallest terms first
              c = mfma_bf16(am, zm, c);
              c = mfma_bf16(ah, zl, c);
              c = mfma_bf16(am, zh, c);
              c = mfma_bf16(ah, zm, c);
              c = mfma_bf16(ah, zh, c);
#pragma unroll
              for (int v = 0; v < 4; ++v) acc64[cb][v] += (double)c[v];
            }
          }
        }
      }
    };
    if (whole && tile * 16 + 16 <= n) chunks(std::true_type{});
    else chunks(std::false_type{});
    double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[v] = fma(acc64[cb][v], acc64[cb][v], sq[v]);
#pragma unroll
    for (int v = 0; v < 4; ++v) sq[v] = sum16(sq[v]);
    if ((lane & 15) == 0) {
      // rows 4 g .. 4 g + 3 of the tile: one 16-byte store when they all
      // exist and theta is 16-byte aligned
      const int64_t r0 = tile * 16 + 4 * g;
      if (theta_vec && r0 + 4 <= n) {
        float4 o = make_float4((float)sq[0], (float)sq[1], (float)sq[2], (float)sq[3]);
        if (ct.acc) {
          const float4 p = *reinterpret_cast<const float4*>(theta + r0);
          o.x += p.x, o.y += p.y, o.z += p.z, o.w += p.w;
        }
        *reinterpret_cast<float4*>(theta + r0) = o;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (r0 + v < n) theta[r0 + v] = ct.acc ? theta[r0 + v] + (float)sq[v] : (float)sq[v];
      }
    }
  }
}

template <int CB, int WG>
hipError_t launch_x3(const float* a, int64_t n, int64_t d, int64_t ld, int64_t nt, const uint4* z, int64_t zvecs,
                     int64_t part_vecs, size_t zbytes, int num_cu, void* theta, const ColTile& ct, hipStream_t s) {
  auto kern = rownorm_x3_kernel<CB, WG>;
  hipError_t e = hipSuccess;
  if (zbytes > 64 * 1024) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)zbytes);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WG, zbytes);
  if (e != hipSuccess) return e;
  const int64_t ntiles = (n + 15) / 16;
  const int64_t want = (ntiles + WG / 64 - 1) / (WG / 64);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * std::max(per_cu, 1)));
  kern<<<(unsigned)blocks, WG, zbytes, s>>>(a, n, d, ld, nt, z, zvecs, part_vecs, theta, ct);
  return hipGetLastError();
}

template <int VAR, typename TA, int CB>
hipError_t launch_cb(const void* A, int64_t n, int64_t d, int64_t ld, int64_t nt, const void* Zpack,
                     size_t zbytes, void* theta, const ColTile& ct, hipStream_t s) {
  using F = Frag<VAR, TA>;
  const int64_t zvecs = (int64_t)(zbytes / 16);
  const int64_t part_vecs = zvecs / F::NZ;
  const int64_t ntiles = (n + 15) / 16;
  const int64_t want = (ntiles + (kThreads / 64) - 1) / (kThreads / 64);
  const TA* a = static_cast<const TA*>(A);
  const uint4* z = static_cast<const uint4*>(Zpack);
  int dev = 0, num_cu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // a persistent grid of exactly the resident workgroups: every wave strides
  // over the 16-row tiles, so no tail of half-empty rounds
  if constexpr (VAR == 4) {
    if (zbytes <= kMaxLdsZ) {
      // (four column tiles need more than the 768-thread shape's 80 registers)
      if constexpr (CB < 4) {
        if (zbytes <= (size_t)X3Shape<768>::kMaxZVecs * 16)
          return launch_x3<CB, 768>(a, n, d, ld, nt, z, zvecs, part_vecs, zbytes, num_cu, theta, ct, s);
      }
      return launch_x3<CB, 1024>(a, n, d, ld, nt, z, zvecs, part_vecs, zbytes, num_cu, theta, ct, s);
    }
  }
  if (zbytes <= kMaxLdsZ) {
    auto kern = rownorm_dense_kernel<VAR, TA, CB, true>;
    if (zbytes > 64 * 1024) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)zbytes);
      if (e != hipSuccess) return e;
    }
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, zbytes);
    if (e != hipSuccess) return e;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * std::max(per_cu, 1)));
    kern<<<(unsigned)blocks, kThreads, zbytes, s>>>(a, n, d, ld, nt, z, zvecs, part_vecs, theta, ct);
  } else {
    auto kern = rownorm_dense_kernel<VAR, TA, CB, false>;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, 0);
    if (e != hipSuccess) return e;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * std::max(per_cu, 1)));
    kern<<<(unsigned)blocks, kThreads, 0, s>>>(a, n, d, ld, nt, z, zvecs, part_vecs, theta, ct);
  }
  return hipGetLastError();
}

template <int VAR, typename TA>
hipError_t launch_var(const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* Zpack,
                      void* theta, const ColTile& ct, hipStream_t s) {
  using F = Frag<VAR, TA>;
  const int64_t nt = (d + F::CW - 1) / F::CW;
  const size_t zbytes = pack_z_operand_bytes(VAR, d, k);
  switch ((k + 15) / 16) {
    case 1: return launch_cb<VAR, TA, 1>(A, n, d, ld, nt, Zpack, zbytes, theta, ct, s);
    case 2: return launch_cb<VAR, TA, 2>(A, n, d, ld, nt, Zpack, zbytes, theta, ct, s);
    case 3: return launch_cb<VAR, TA, 3>(A, n, d, ld, nt, Zpack, zbytes, theta, ct, s);
    case 4: return launch_cb<VAR, TA, 4>(A, n, d, ld, nt, Zpack, zbytes, theta, ct, s);
    default: return hipErrorInvalidValue;
  }
}

// One column tile (k <= 64) of pass 2.
hipError_t launch_tile(int variant, int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k,
                       const void* Zpack, void* theta, const ColTile& ct, hipStream_t s) {
  if (variant == 0 && dtype == 0) return launch_var<0, double>(A, n, d, ld, k, Zpack, theta, ct, s);
  if (variant == 1 && dtype == 1) return launch_var<1, float>(A, n, d, ld, k, Zpack, theta, ct, s);
  if (variant == 1 && dtype == 2) return launch_var<1, __hip_bfloat16>(A, n, d, ld, k, Zpack, theta, ct, s);
  // BF16 storage: the streaming kernel of rownorm_bf16.hip, Z in 1, 2 or 3 parts
  if (variant == 2 && dtype == 2) return launch_rownorm_bf16(1, A, n, d, ld, k, Zpack, theta, ct, s);
  if (variant == 3 && dtype == 2) return launch_rownorm_bf16(2, A, n, d, ld, k, Zpack, theta, ct, s);
  if (variant == 4 && dtype == 2) return launch_rownorm_bf16(3, A, n, d, ld, k, Zpack, theta, ct, s);
  if (variant == 4 && dtype == 1) return launch_var<4, float>(A, n, d, ld, k, Zpack, theta, ct, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_rownorm_dense(int variant, int dtype, const void* A, int64_t n, int64_t d, int64_t ld,
                                int64_t k, const void* Zpack, const int64_t* live, void* theta,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // k > 64: one pass over A per column tile of 64, each adding its squares
  // to theta (the first stores); a tile past the live columns returns at once
  for (int64_t t = 0; t < z_tiles(k); ++t) {
    ColTile ct;
    ct.c0 = t * kZTile;
    ct.acc = t > 0;
    ct.live = t > 0 ? live : nullptr;
    const int64_t kt = std::min<int64_t>(kZTile, k - ct.c0);
    const void* zt = static_cast<const char*>(Zpack) + pack_z_tile_offset(variant, d, k, t);
    hipError_t e = launch_tile(variant, dtype, A, n, d, ld, kt, zt, theta, ct, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lev
