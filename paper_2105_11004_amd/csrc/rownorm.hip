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
// may be stored as FP32 or BF16), BF16 (16x16x32bf16, EL 8, Z in BF16) and
// BF16 hi/lo (two BF16 products, Z = Z_hi + Z_lo).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lev_internal.h"

namespace lev {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---- per-variant traits ----------------------------------------------------
// Load one lane's A fragment for chunk t; returns it in the MFMA input type.
template <int VAR, typename TA>
struct Frag;

// FP64: two doubles per lane, 16-byte load.
template <>
struct Frag<0, double> {
  static constexpr int EL = 2, CW = 8;
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
  static constexpr int EL = 4, CW = 16;
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
  static constexpr int EL = 4, CW = 16;
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

// BF16: eight bf16, 16-byte load.
template <int VAR>
struct FragBf16 {
  static constexpr int EL = 8, CW = 32;
  using T = uint4;
  __device__ static T load(const __hip_bfloat16* row, int64_t col, int64_t d, bool ok) {
    if (!ok || col >= d) return make_uint4(0u, 0u, 0u, 0u);
    uint4 v = *reinterpret_cast<const uint4*>(row + col);
    if (col + 7 >= d) {
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (col + e >= d) w[e >> 1] &= (e & 1) ? 0x0000FFFFu : 0xFFFF0000u;
      v = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return v;
  }
};
template <>
struct Frag<2, __hip_bfloat16> : FragBf16<2> {};
template <>
struct Frag<3, __hip_bfloat16> : FragBf16<3> {};

template <int VAR>
struct Acc {
  using T = v4f;
};
template <>
struct Acc<0> {
  using T = v4d;
};

// acc += A_frag * Z_frag over one chunk of the contraction.
template <int VAR>
__device__ __forceinline__ void mma(typename Acc<VAR>::T& acc, const uint4& a, const uint4& b,
                                    const uint4& b_lo);

template <>
__device__ __forceinline__ void mma<0>(v4d& acc, const uint4& a, const uint4& b, const uint4&) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double((int)a.y, (int)a.x),
                                             __hiloint2double((int)b.y, (int)b.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double((int)a.w, (int)a.z),
                                             __hiloint2double((int)b.w, (int)b.z), acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<1>(v4f& acc, const uint4& a, const uint4& b, const uint4&) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<2>(v4f& acc, const uint4& a, const uint4& b, const uint4&) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<3>(v4f& acc, const uint4& a, const uint4& b, const uint4& b_lo) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                __builtin_bit_cast(v8bf, b_lo), acc, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T sum16(T x) {
  // reduce over the 16 lanes sharing l / 16 (xor over the low 4 bits)
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

constexpr int kThreads = 256;
constexpr int kBatch = 8;  // chunks loaded per batch (loads in flight per lane)

// Zpack: ((t*CB + cb)*64 + l) 16-byte vectors (BF16 hi/lo: lo part follows
// the hi part, `lo_off` vectors later).
template <int VAR, typename TA, int CB, bool ZLDS>
__global__ __launch_bounds__(kThreads) void rownorm_dense_kernel(const TA* __restrict__ A, int64_t n,
                                                                 int64_t d, int64_t ld, int64_t nt,
                                                                 const uint4* __restrict__ Zg,
                                                                 int64_t zvecs, int64_t lo_off,
                                                                 void* __restrict__ theta) {
  using F = Frag<VAR, TA>;
  using AccT = typename Acc<VAR>::T;
  extern __shared__ uint4 zs[];
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
    // every chunk, so FP32 rounding only ever sums one chunk's products.
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
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int64_t zi = (t * CB + cb) * 64 + lane;
            const uint4 b = Z[zi];
            uint4 blo = make_uint4(0u, 0u, 0u, 0u);
            if constexpr (VAR == 3) blo = Z[zi + lo_off];
            mma<VAR>(acc[cb], a[u], b, blo);
          }
          if constexpr (VAR != 0) {
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
          if constexpr (VAR == 0) static_cast<double*>(theta)[r] = s[v];
          else static_cast<float*>(theta)[r] = (float)s[v];
        }
      }
    }
  }
}

template <int VAR, typename TA, int CB>
hipError_t launch_cb(const void* A, int64_t n, int64_t d, int64_t ld, int64_t nt, const void* Zpack,
                     size_t zbytes, void* theta, hipStream_t s) {
  const int64_t zvecs = (int64_t)(zbytes / 16);
  const int64_t lo_off = (VAR == 3) ? zvecs / 2 : 0;
  const int64_t ntiles = (n + 15) / 16;
  int64_t blocks = (ntiles + 3) / 4;
  const int64_t max_blocks = 256 * 8;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  const TA* a = static_cast<const TA*>(A);
  const uint4* z = static_cast<const uint4*>(Zpack);
  if (zbytes <= 64 * 1024) {
    rownorm_dense_kernel<VAR, TA, CB, true><<<(unsigned)blocks, kThreads, zbytes, s>>>(
        a, n, d, ld, nt, z, zvecs, lo_off, theta);
  } else {
    rownorm_dense_kernel<VAR, TA, CB, false><<<(unsigned)blocks, kThreads, 0, s>>>(a, n, d, ld, nt, z, zvecs,
                                                                                   lo_off, theta);
  }
  return hipGetLastError();
}

template <int VAR, typename TA>
hipError_t launch_var(const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* Zpack,
                      void* theta, hipStream_t s) {
  using F = Frag<VAR, TA>;
  const int64_t nt = (d + F::CW - 1) / F::CW;
  const size_t zbytes = pack_z_bytes(VAR, d, k);
  switch ((k + 15) / 16) {
    case 1: return launch_cb<VAR, TA, 1>(A, n, d, ld, nt, Zpack, zbytes, theta, s);
    case 2: return launch_cb<VAR, TA, 2>(A, n, d, ld, nt, Zpack, zbytes, theta, s);
    case 3: return launch_cb<VAR, TA, 3>(A, n, d, ld, nt, Zpack, zbytes, theta, s);
    case 4: return launch_cb<VAR, TA, 4>(A, n, d, ld, nt, Zpack, zbytes, theta, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_rownorm_dense(int variant, int dtype, const void* A, int64_t n, int64_t d, int64_t ld,
                                int64_t k, const void* Zpack, const int64_t* rank, void* theta,
                                hipStream_t s) {
  (void)rank;
  if (n <= 0) return hipSuccess;
  if (variant == 0 && dtype == 0) return launch_var<0, double>(A, n, d, ld, k, Zpack, theta, s);
  if (variant == 1 && dtype == 1) return launch_var<1, float>(A, n, d, ld, k, Zpack, theta, s);
  if (variant == 1 && dtype == 2) return launch_var<1, __hip_bfloat16>(A, n, d, ld, k, Zpack, theta, s);
  if (variant == 2 && dtype == 2) return launch_var<2, __hip_bfloat16>(A, n, d, ld, k, Zpack, theta, s);
  if (variant == 3 && dtype == 2) return launch_var<3, __hip_bfloat16>(A, n, d, ld, k, Zpack, theta, s);
  return hipErrorInvalidValue;
}

}  // namespace lev
