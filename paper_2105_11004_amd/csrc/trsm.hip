// Algorithm 8, step 4, on the selected columns: X = R~^{-1} Pi_2, here
// Z = R11^{-1} G_k[0:r, :] by back substitution in FP64 (R11 is the leading
// r x r block of the pivoted factor; r is read on the device), then Z is
// scattered to the original column ids (Z_full[perm[j], :] = Z[j, :], zero
// rows off K) and converted to the operand layout of pass 2.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Pass-2 operand layouts (see rownorm.hip).  For chunk t of the contraction
// (CW columns), column tile cb (16 output columns), lane l and element e:
//   value = Z_full[t*CW + EL*(l/16) + e][16*cb + (l%16)]
// stored at ((t*CB + cb)*64 + l)*EL + e, CB = ceil(k/16).
//   FP64: EL = 2, CW = 8.   FP32: EL = 4, CW = 16.   BF16: EL = 8, CW = 32.
template <typename OUT, int EL>
__global__ void pack_z_kernel(int64_t d, int64_t k, const int32_t* __restrict__ perm,
                              const int64_t* __restrict__ rank, const double* __restrict__ Z64,
                              OUT* __restrict__ out, OUT* __restrict__ out_lo, int64_t nt, int64_t cbn) {
  constexpr int CW = 4 * EL;
  const int64_t total = nt * cbn * 64 * EL;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % EL);
  const int l = (int)((idx / EL) % 64);
  const int64_t cb = (idx / (EL * 64)) % cbn;
  const int64_t t = idx / (EL * 64 * cbn);
  const int64_t row = t * CW + EL * (l / 16) + e;  // original column id of A
  const int64_t col = 16 * cb + (l % 16);
  const int64_t r = *rank;
  double v = 0.0;
  if (row < d && col < k) {
    // position of column `row` among the pivots (linear scan; d <= 1024)
    for (int64_t j = 0; j < r; ++j) {
      if (perm[j] == row) {
        v = Z64[j * k + col];
        break;
      }
    }
  }
  if constexpr (sizeof(OUT) == 2) {
    const __hip_bfloat16 hi = __double2bfloat16(v);
    out[idx] = hi;
    if (out_lo != nullptr) out_lo[idx] = __double2bfloat16(v - (double)__bfloat162float(hi));
  } else {
    out[idx] = (OUT)v;
  }
}

constexpr int64_t chunk_cols(int variant) { return variant == 0 ? 8 : (variant == 1 ? 16 : 32); }

}  // namespace

hipError_t launch_trsm_z(int64_t d, int64_t k, const double* R, const int64_t* rank, const double* Gk,
                         double* Z64, hipStream_t s) {
  trsm_z_kernel<<<(unsigned)k, 64, (size_t)d * sizeof(double), s>>>(d, k, R, rank, Gk, Z64);
  return hipGetLastError();
}

size_t pack_z_bytes(int variant, int64_t d, int64_t k) {
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
  const int64_t elems = nt * cbn * 64 * (cw / 4);
  switch (variant) {
    case 0: return (size_t)elems * 8;
    case 1: return (size_t)elems * 4;
    case 2: return (size_t)elems * 2;
    case 3: return (size_t)elems * 4;  // hi then lo
    default: return 0;
  }
}

hipError_t launch_pack_z(int variant, int64_t d, int64_t k, const int32_t* perm, const int64_t* rank,
                         const double* Z64, void* Zpack, hipStream_t s) {
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
  const int64_t total = nt * cbn * 64 * (cw / 4);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  switch (variant) {
    case 0:
      pack_z_kernel<double, 2><<<blocks, 256, 0, s>>>(d, k, perm, rank, Z64, static_cast<double*>(Zpack),
                                                      nullptr, nt, cbn);
      break;
    case 1:
      pack_z_kernel<float, 4><<<blocks, 256, 0, s>>>(d, k, perm, rank, Z64, static_cast<float*>(Zpack),
                                                     nullptr, nt, cbn);
      break;
    case 2:
      pack_z_kernel<__hip_bfloat16, 8><<<blocks, 256, 0, s>>>(
          d, k, perm, rank, Z64, static_cast<__hip_bfloat16*>(Zpack), nullptr, nt, cbn);
      break;
    case 3: {
      __hip_bfloat16* hi = static_cast<__hip_bfloat16*>(Zpack);
      pack_z_kernel<__hip_bfloat16, 8><<<blocks, 256, 0, s>>>(d, k, perm, rank, Z64, hi, hi + total, nt,
                                                              cbn);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lev
