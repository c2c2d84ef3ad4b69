// Algorithm 8, step 4, on the selected columns: X = R~^{-1} Pi_2, here
// Z = R11^{-1} G_k[0:r, :] by back substitution in FP64 (R11 is the leading
// r x r block of the pivoted factor; r is read on the device), then Z is
// scattered to the original column ids (Z_full[perm[j], :] = Z[j, :], zero
// rows off K) and converted to the operand layout of pass 2.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lev_internal.h"

namespace lev {
namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// One 64-thread workgroup per right-hand side c < k.  The dot product of
// row j of R with the solved tail is split over the 64 lanes; the next row
// is prefetched while the current one is reduced.
__global__ __launch_bounds__(64) void trsm_z_kernel(int64_t d, int64_t k, const double* __restrict__ R,
                                                    const int64_t* __restrict__ rank,
                                                    const double* __restrict__ Gk,
                                                    double* __restrict__ Z64) {
  extern __shared__ double zs[];  // d entries
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t r = *rank;
  for (int64_t j = r + lane; j < d; j += 64) Z64[j * k + c] = 0.0;
  for (int64_t j = r - 1; j >= 0; --j) {
    double part = 0.0;
    for (int64_t t = j + 1 + lane; t < r; t += 64) part = fma(R[j * d + t], zs[t], part);
    const double tot = wave_sum(part);
    const double zj = (Gk[j * k + c] - tot) / R[j * d + j];
    if (lane == 0) {
      zs[j] = zj;
      Z64[j * k + c] = zj;
    }
    __syncthreads();
  }
}

// r <= 256: one workgroup of 16 waves per group of 64 right-hand sides
// (grid.y).  Wave w holds row block w (rows 16 w .. 16 w + 15) of the
// right-hand side, lane c column c, in registers.  Blocked back
// substitution from the last block: the owner wave of block b solves its
// 16 x 16 diagonal triangle in-lane (no cross-lane traffic), publishes the
// block of Z through LDS, and every wave above applies the 16 x 16 update
// G_w -= R[w, b] Z_b.  R's 16-column panel of block b is staged in LDS
// (double-buffered), so the loop reads no global memory; r / 16 block steps
// instead of r row steps.
constexpr int kTrsmR = 256;
typedef double v16d __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(1024) void trsm_blocked_kernel(int64_t d, int64_t k, const double* __restrict__ R,
                                                            const int64_t* __restrict__ rank,
                                                            const double* __restrict__ Gk,
                                                            double* __restrict__ Z64) {
  __shared__ double rpan[2][kTrsmR][16];  // 64 KB: R[0:r, 16 b .. 16 b + 15]
  __shared__ double zblk[2][16][64];      // the block of Z just solved
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t c = (int64_t)blockIdx.y * 64 + lane;
  const int r = (int)*rank;
  const bool col_ok = c < k;

  v16d g;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = 16 * w + s;
    g[s] = (col_ok && t < r) ? Gk[(int64_t)t * k + c] : 0.0;
  }
  for (int64_t t = r + w; t < d; t += 16)
    if (col_ok) Z64[t * k + c] = 0.0;
  if (r == 0) return;

  auto stage = [&](int blk, int buf) {
    const int rows = 16 * (blk + 1);  // rows 0 .. 16 blk + 15 use this panel
    for (int e = threadIdx.x; e < rows * 16; e += blockDim.x) {
      const int t = e / 16, cc = e % 16;
      const int col = 16 * blk + cc;
      rpan[buf][t][cc] = (t < r && col < r) ? R[(int64_t)t * d + col] : 0.0;
    }
  };
  const int nblk = (r + 15) / 16;
  stage(nblk - 1, (nblk - 1) & 1);
  __syncthreads();
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int buf = blk & 1;
    if (w == blk) {
      // rows past the rank stay zero (R has zero rows there)
#pragma unroll
      for (int s = 15; s >= 0; --s) {
        double x = g[s];
#pragma unroll
        for (int e = s + 1; e < 16; ++e) x = fma(-rpan[buf][16 * blk + s][e], g[e], x);
        g[s] = (16 * blk + s < r) ? x / rpan[buf][16 * blk + s][s] : 0.0;
        zblk[buf][s][lane] = g[s];
      }
    }
    if (blk > 0) stage(blk - 1, buf ^ 1);
    __syncthreads();
    if (w < blk) {
      double z[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) z[e] = zblk[buf][e][lane];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        double x = g[s];
#pragma unroll
        for (int e = 0; e < 16; ++e) x = fma(-rpan[buf][16 * w + s][e], z[e], x);
        g[s] = x;
      }
    }
    __syncthreads();  // rpan[buf] and zblk[buf] are rewritten two steps later
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = 16 * w + s;
    if (col_ok && t < r) Z64[(int64_t)t * k + c] = g[s];
  }
}

// Pass-2 operand layouts (see rownorm.hip).  For chunk t of the contraction
// (CW columns), column tile cb (16 output columns), lane l and element e:
//   value = Z_full[t*CW + EL*(l/16) + e][16*cb + (l%16)]
// stored at ((t*CB + cb)*64 + l)*EL + e, CB = ceil(k/16).
//   FP64: EL = 2, CW = 8.   FP32: EL = 4, CW = 16.   BF16 forms: EL = 8, CW = 32.
// BF16 forms store NP parts one after the other: part 0 = RNE(v), part p =
// RNE(v - parts 0..p-1) (NP = 1 BF16, 2 BF16 hi/lo, 3 BF16x3).
// Value of packed element idx (see the layout above); inv maps a column id
// to its pivot position (-1 off K), Z64 is r x k by pivot position.
// (32-bit index arithmetic: the operand has at most 2^18 elements.)
template <typename OUT, int EL, int NP>
__device__ __forceinline__ void pack_element(int idx, int total, int d, int k, int cbn, const int32_t* inv,
                                             const double* __restrict__ Z64, OUT* out) {
  constexpr int CW = 4 * EL;
  const int e = idx % EL;
  const int l = (idx / EL) % 64;
  const int q = idx / (EL * 64);
  const int cb = q % cbn;
  const int t = q / cbn;
  const int row = t * CW + EL * (l / 16) + e;  // original column id of A
  const int col = 16 * cb + (l % 16);
  double v = 0.0;
  if (row < d && col < k) {
    const int32_t j = inv[row];  // pivot position, or -1 when not selected
    if (j >= 0) v = Z64[(int64_t)j * k + col];
  }
  if constexpr (sizeof(OUT) == 2) {
    double rest = v;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const __hip_bfloat16 part = __double2bfloat16(rest);
      out[p * total + idx] = part;
      rest -= (double)__bfloat162float(part);
    }
  } else {
    out[idx] = (OUT)v;
  }
}

template <typename OUT, int EL, int NP>
__global__ void pack_z_kernel(int64_t d, int64_t k, const int32_t* __restrict__ inv_perm,
                              const double* __restrict__ Z64, OUT* __restrict__ out, int64_t nt,
                              int64_t cbn) {
  const int total = (int)(nt * cbn * 64 * EL);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  pack_element<OUT, EL, NP>(idx, total, (int)d, (int)k, (int)cbn, inv_perm, Z64, out);
}

// CSR operand value of element idx of the d x 64 row-major Z_full.
template <typename OUT>
__device__ __forceinline__ void pack_rowmajor_element(int idx, int k, const int32_t* inv,
                                                      const double* __restrict__ Z64, OUT* out) {
  const int row = idx / 64, col = idx % 64;
  double v = 0.0;
  if (col < k) {
    const int32_t j = inv[row];
    if (j >= 0) v = Z64[(int64_t)j * k + col];
  }
  out[idx] = (OUT)v;
}

// inv_perm[c] = pivot position of column c (-1 when c is not among the r
// selected columns).
__global__ void inverse_perm_kernel(int64_t d, const int32_t* __restrict__ perm, const int64_t* __restrict__ rank,
                                    int32_t* __restrict__ inv_perm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const int64_t r = *rank;
  inv_perm[perm[j]] = j < r ? (int32_t)j : -1;
}

// CSR operand: Z_full row-major with rows padded to 64 columns.
template <typename OUT>
__global__ void pack_z_rowmajor_kernel(int64_t d, int64_t k, const int32_t* __restrict__ inv_perm,
                                       const double* __restrict__ Z64, OUT* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * 64) return;
  pack_rowmajor_element<OUT>(idx, (int)k, inv_perm, Z64, out);
}

constexpr int64_t chunk_cols(int variant) { return variant == 0 ? 8 : (variant == 1 ? 16 : 32); }
constexpr int parts(int variant) { return variant == 3 ? 2 : (variant == 4 ? 3 : 1); }

// Z = R11^{-1} G_k, then Z_full packed for pass 2, in one workgroup (r <= 256,
// k <= 64): the blocked back substitution of trsm_blocked_kernel with the R
// panel of the next block prefetched into registers during the current
// block's solve, Z stored (state), the inverse permutation built in LDS and
// the packed operand written from the just-stored Z (L2-resident).
template <int VARIANT>
__global__ __launch_bounds__(1024) void form_z_kernel(int64_t d, int64_t k, const double* __restrict__ R,
                                                      const int64_t* __restrict__ rank,
                                                      const int32_t* __restrict__ perm,
                                                      const double* __restrict__ Gk, double* __restrict__ Z64,
                                                      void* __restrict__ Zpack, int64_t nt, int64_t cbn) {
  __shared__ double rpan[2][kTrsmR][16];  // 64 KB: R[0:r, 16 b .. 16 b + 15]
  __shared__ double zblk[2][16][64];      // the block of Z just solved
  __shared__ int32_t inv[kTrsmR];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane;
  const int r = (int)*rank;
  const bool col_ok = c < k;

  v16d g;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = 16 * w + s;
    g[s] = (col_ok && t < r) ? Gk[(int64_t)t * k + c] : 0.0;
  }
  for (int64_t t = r + w; t < d; t += 16)
    if (col_ok) Z64[t * k + c] = 0.0;
  for (int j = threadIdx.x; j < d; j += blockDim.x) inv[perm[j]] = j < r ? j : -1;

  // panel b: rows 0 .. 16 b + 15 of columns 16 b .. 16 b + 15 (4 per thread)
  double pre[4];
  auto load_panel = [&](int blk) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 1024 * q;
      const int t = e / 16, cc = e % 16;
      const int col = 16 * blk + cc;
      pre[q] = (t < 16 * (blk + 1) && t < r && col < r) ? R[(int64_t)t * d + col] : 0.0;
    }
  };
  auto store_panel = [&](int blk) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 1024 * q;
      rpan[blk & 1][e / 16][e % 16] = pre[q];
    }
  };
  const int nblk = (r + 15) / 16;
  if (nblk > 0) {
    load_panel(nblk - 1);
    store_panel(nblk - 1);
    if (nblk > 1) load_panel(nblk - 2);
  }
  __syncthreads();
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int buf = blk & 1;
    if (w == blk) {
#pragma unroll
      for (int s = 15; s >= 0; --s) {
        double x = g[s];
#pragma unroll
        for (int e = s + 1; e < 16; ++e) x = fma(-rpan[buf][16 * blk + s][e], g[e], x);
        g[s] = (16 * blk + s < r) ? x / rpan[buf][16 * blk + s][s] : 0.0;
        zblk[buf][s][lane] = g[s];
      }
    }
    if (blk > 0) {
      store_panel(blk - 1);  // loaded during the previous block
      if (blk > 1) load_panel(blk - 2);
    }
    __syncthreads();
    if (w < blk) {
      double z[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) z[e] = zblk[buf][e][lane];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        double x = g[s];
#pragma unroll
        for (int e = 0; e < 16; ++e) x = fma(-rpan[buf][16 * w + s][e], z[e], x);
        g[s] = x;
      }
    }
    __syncthreads();  // rpan[buf] and zblk[buf] are rewritten two steps later
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = 16 * w + s;
    if (col_ok && t < r) Z64[(int64_t)t * k + c] = g[s];
  }
  __syncthreads();  // Z64 and inv visible to the whole workgroup
  // eight elements per thread and round, so their reads of Z overlap
  constexpr int U = 8;
  const int di = (int)d, ki = (int)k;
  if constexpr (VARIANT == 5 || VARIANT == 6) {
    using OUT = typename std::conditional<VARIANT == 5, float, double>::type;
    for (int i0 = threadIdx.x; i0 < di * 64; i0 += 1024 * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = i0 + 1024 * u;
        if (idx < di * 64) pack_rowmajor_element<OUT>(idx, ki, inv, Z64, static_cast<OUT*>(Zpack));
      }
    }
  } else {
    constexpr int EL = VARIANT == 0 ? 2 : (VARIANT == 1 ? 4 : 8);
    constexpr int NP = VARIANT == 3 ? 2 : (VARIANT == 4 ? 3 : 1);
    using OUT = typename std::conditional<VARIANT == 0, double,
                typename std::conditional<VARIANT == 1, float, __hip_bfloat16>::type>::type;
    const int total = (int)(nt * cbn * 64 * EL);
    const int cbi = (int)cbn;
    for (int i0 = threadIdx.x; i0 < total; i0 += 1024 * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = i0 + 1024 * u;
        if (idx < total) pack_element<OUT, EL, NP>(idx, total, di, ki, cbi, inv, Z64, static_cast<OUT*>(Zpack));
      }
    }
  }
}

}  // namespace

hipError_t launch_trsm_z(int64_t d, int64_t k, const double* R, const int64_t* rank, const double* Gk,
                         double* Z64, hipStream_t s) {
  if (d <= kTrsmR) {
    trsm_blocked_kernel<<<dim3(1, (unsigned)((k + 63) / 64)), 1024, 0, s>>>(d, k, R, rank, Gk, Z64);
  } else {
    trsm_z_kernel<<<(unsigned)k, 64, (size_t)d * sizeof(double), s>>>(d, k, R, rank, Gk, Z64);
  }
  return hipGetLastError();
}

size_t pack_z_operand_bytes(int variant, int64_t d, int64_t k) {
  if (variant == 5 || variant == 6) return (size_t)d * 64 * (variant == 5 ? 4 : 8);
  if (variant < 0 || variant > 4) return 0;
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
  const int64_t elems = nt * cbn * 64 * (cw / 4);
  const size_t esize = variant == 0 ? 8 : (variant == 1 ? 4 : 2);
  return (size_t)elems * esize * (size_t)parts(variant);
}

size_t pack_z_bytes(int variant, int64_t d, int64_t k) {
  if (variant < 0 || variant > 6) return 0;
  return pack_z_operand_bytes(variant, d, k) + (size_t)d * sizeof(int32_t);
}

// Zpack layout: the packed operand (as above) followed by inv_perm[d].
hipError_t launch_pack_z(int variant, int64_t d, int64_t k, const int32_t* perm, const int64_t* rank,
                         const double* Z64, void* Zpack, hipStream_t s) {
  if (variant == 5 || variant == 6) {
    int32_t* inv = reinterpret_cast<int32_t*>(static_cast<char*>(Zpack) + pack_z_operand_bytes(variant, d, k));
    inverse_perm_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, perm, rank, inv);
    const unsigned blocks = (unsigned)((d * 64 + 255) / 256);
    if (variant == 5)
      pack_z_rowmajor_kernel<float><<<blocks, 256, 0, s>>>(d, k, inv, Z64, static_cast<float*>(Zpack));
    else
      pack_z_rowmajor_kernel<double><<<blocks, 256, 0, s>>>(d, k, inv, Z64, static_cast<double*>(Zpack));
    return hipGetLastError();
  }
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
  const int64_t total = nt * cbn * 64 * (cw / 4);
  const size_t esize = variant == 0 ? 8 : (variant == 1 ? 4 : 2);
  int32_t* inv = reinterpret_cast<int32_t*>(static_cast<char*>(Zpack) + (size_t)total * esize * parts(variant));
  inverse_perm_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, perm, rank, inv);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  switch (variant) {
    case 0:
      pack_z_kernel<double, 2, 1><<<blocks, 256, 0, s>>>(d, k, inv, Z64, static_cast<double*>(Zpack), nt, cbn);
      break;
    case 1:
      pack_z_kernel<float, 4, 1><<<blocks, 256, 0, s>>>(d, k, inv, Z64, static_cast<float*>(Zpack), nt, cbn);
      break;
    case 2:
      pack_z_kernel<__hip_bfloat16, 8, 1><<<blocks, 256, 0, s>>>(d, k, inv, Z64,
                                                                 static_cast<__hip_bfloat16*>(Zpack), nt, cbn);
      break;
    case 3:
      pack_z_kernel<__hip_bfloat16, 8, 2><<<blocks, 256, 0, s>>>(d, k, inv, Z64,
                                                                 static_cast<__hip_bfloat16*>(Zpack), nt, cbn);
      break;
    case 4:
      pack_z_kernel<__hip_bfloat16, 8, 3><<<blocks, 256, 0, s>>>(d, k, inv, Z64,
                                                                 static_cast<__hip_bfloat16*>(Zpack), nt, cbn);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_form_z(int variant, int64_t d, int64_t k, const double* R, const int64_t* rank,
                         const int32_t* perm, const double* Gk, double* Z64, void* Zpack, hipStream_t s) {
  if (variant < 0 || variant > 6) return hipErrorInvalidValue;
  if (d > kTrsmR || k > 64) {
    hipError_t e = launch_trsm_z(d, k, R, rank, Gk, Z64, s);
    if (e != hipSuccess) return e;
    return launch_pack_z(variant, d, k, perm, rank, Z64, Zpack, s);
  }
  const int64_t cw = variant >= 5 ? 1 : chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
#define LEV_FZ(V)                                                                                      \
  case V:                                                                                              \
    form_z_kernel<V><<<1, 1024, 0, s>>>(d, k, R, rank, perm, Gk, Z64, Zpack, nt, cbn);                  \
    break;
  switch (variant) {
    LEV_FZ(0) LEV_FZ(1) LEV_FZ(2) LEV_FZ(3) LEV_FZ(4) LEV_FZ(5) LEV_FZ(6)
  }
#undef LEV_FZ
  return hipGetLastError();
}

}  // namespace lev
