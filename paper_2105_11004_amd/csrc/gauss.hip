// Gaussian matrices of the estimator (Section 3.4, Gaussian embeddings):
// G_m / sqrt(m) of Algorithm 3 and the JL Gaussian Pi_2 / sqrt(k) of
// Algorithm 8.  Element e (row-major) uses Philox4x32-10 counter floor(e/2);
// the two uniforms of that counter feed Box-Muller, whose cosine branch is
// element 2q and sine branch element 2q+1.  Also the zero-fill helper.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_device.h"
#include "lev_internal.h"

namespace lev {
namespace {

__global__ void gaussian_kernel(PhiloxKey key, int64_t total, double scale, double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = 2 * q;
  if (e >= total) return;
  double z0, z1;
  box_muller_pair((uint64_t)q, key, &z0, &z1);
  out[e] = z0 * scale;
  if (e + 1 < total) out[e + 1] = z1 * scale;
}

__global__ void fill_zero_kernel(uint4* __restrict__ p, size_t n16, uint8_t* __restrict__ tail,
                                 size_t ntail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = i; j < n16; j += stride) p[j] = make_uint4(0u, 0u, 0u, 0u);
  if (i < ntail) tail[i] = 0;
}

__global__ void store_i64x4_kernel(int64_t* dst, int64_t a, int64_t b, int64_t c, int64_t e) {
  if (threadIdx.x == 0) {
    dst[0] = a;
    dst[1] = b;
    dst[2] = c;
    dst[3] = e;
  }
}

}  // namespace

hipError_t launch_store_i64x4(int64_t* dst, int64_t a, int64_t b, int64_t c, int64_t e, hipStream_t s) {
  store_i64x4_kernel<<<1, 64, 0, s>>>(dst, a, b, c, e);
  return hipGetLastError();
}

hipError_t launch_gaussian(PhiloxKey key, int64_t rows, int64_t cols, double scale, double* out,
                           hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  const int64_t pairs = (total + 1) / 2;
  gaussian_kernel<<<(unsigned)((pairs + 255) / 256), 256, 0, s>>>(key, total, scale, out);
  return hipGetLastError();
}

// Zeroes `bytes` bytes at p (p 16-byte aligned).  A kernel rather than
// hipMemsetAsync so that a stream capture records an ordinary kernel node.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  const size_t blocks = std::min<size_t>(4096, (n16 + 255) / 256 + 1);
  fill_zero_kernel<<<(unsigned)blocks, 256, 0, s>>>(static_cast<uint4*>(p), n16,
                                                    static_cast<uint8_t*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace lev
