// The SRHT of Section 3.4 applied to the CountSketch's output (the F S
// composition of Section 4): A~ = F (S A) with F = sqrt(r / t) P (H / sqrt(r))
// D = P H D / sqrt(t), H the unscaled r x r Walsh-Hadamard matrix (Sylvester
// order, r a power of two), D = diag(+-1) and P the first t coordinates of a
// keyed permutation pi of [0, r).  It takes the place of the t x r x d
// Gaussian product: H costs r d log2(r) additions.
//
// Conventions (the definitions the oracle implements on its own):
//   D_jj = -1 iff bit 63 of mix64(key_d + j gamma) is set;
//   pi: a four-round Feistel network on 2h-bit words (h = max(1,
//   ceil(log2(r) / 2))), round t's function mix64(key_p + (t 2^32 + right)
//   gamma) mod 2^h, walked along its cycle until the value is < r;
// with mix64 the SplitMix64 finaliser and gamma = 0x9E3779B97F4A7C15.
//
// H runs as radix-2^nb passes (nb <= 8) over the row index of the FP64
// S A (r x d, row-major, transformed in place): pass q handles bits
// [b0, b0 + nb), a workgroup loads the 2^nb rows base + u 2^b0 of 32
// columns into LDS, does the nb butterfly stages (a, b) -> (a + b, a - b)
// and writes them back.  The first pass multiplies by D on the load; the
// last writes only the sampled rows, row pi(j) to row j of A~, times
// 1 / sqrt(t).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kMaxBits = 8;   // rows per group: 2^8
constexpr int kCols = 32;     // columns per workgroup
constexpr int kThreads = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t feistel(uint64_t key, uint64_t x, int h) {
  const uint64_t mask = (1ull << h) - 1;
  uint64_t left = x >> h, right = x & mask;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint64_t f = mix64(key + (((uint64_t)t << 32) + right) * kGamma) & mask;
    const uint64_t nl = right;
    right = left ^ f;
    left = nl;
  }
  return (left << h) | right;
}

// inv[pi(j)] = j for j < t (the other entries were set to -1 before).
// Cycle walking ends: pi is a permutation of [0, 2^{2h}) and j < r.
__global__ void srht_sample_kernel(uint64_t key_p, int64_t r, int64_t t, int h, int32_t* __restrict__ inv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= t) return;
  uint64_t y = feistel(key_p, (uint64_t)j, h);
  while (y >= (uint64_t)r) y = feistel(key_p, y, h);
  inv[y] = (int32_t)j;
}

__global__ void fill_minus_one_kernel(int64_t r, int32_t* __restrict__ inv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < r) inv[j] = -1;
}

__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// One radix-2^nb pass of H over bits [b0, b0 + nb) of the row index.
__global__ __launch_bounds__(kThreads) void fwht_pass_kernel(double* __restrict__ X, int64_t r, int64_t d, int b0,
                                                             int nb, int first, uint64_t key_d, int last,
                                                             const int32_t* __restrict__ inv, double scale,
                                                             double* __restrict__ At) {
  __shared__ double T[(1 << kMaxBits) * kCols];
  const int G = 1 << nb;
  const int64_t g = blockIdx.x;  // group: low bits (below b0) and high bits (above b0 + nb) of the rows
  const int64_t low = g & ((1ll << b0) - 1);
  const int64_t base = ((g >> b0) << (b0 + nb)) | low;
  const int64_t stride = 1ll << b0;
  const int64_t c0 = (int64_t)blockIdx.y * kCols;
  const int tid = threadIdx.x;
  for (int e = tid; e < G * kCols; e += kThreads) {
    const int u = e / kCols, c = e % kCols;
    const int64_t row = base + u * stride, col = c0 + c;
    double v = col < d ? X[row * d + col] : 0.0;
    if (first && (mix64(key_d + (uint64_t)row * kGamma) >> 63)) v = -v;
    T[e] = v;
  }
  lds_barrier();
  for (int s = 0; s < nb; ++s) {
    for (int q = tid; q < (G / 2) * kCols; q += kThreads) {
      const int c = q % kCols, pu = q / kCols;
      const int u0 = ((pu >> s) << (s + 1)) | (pu & ((1 << s) - 1));
      const int u1 = u0 | (1 << s);
      const double a = T[u0 * kCols + c], b = T[u1 * kCols + c];
      T[u0 * kCols + c] = a + b;
      T[u1 * kCols + c] = a - b;
    }
    lds_barrier();
  }
  for (int e = tid; e < G * kCols; e += kThreads) {
    const int u = e / kCols, c = e % kCols;
    const int64_t row = base + u * stride, col = c0 + c;
    if (col >= d) continue;
    if (last) {
      const int32_t j = inv[row];
      if (j >= 0) At[(int64_t)j * d + col] = T[e] * scale;
    } else {
      X[row * d + col] = T[e];
    }
  }
}

}  // namespace

hipError_t launch_srht(uint64_t key_d, uint64_t key_p, int64_t r, int64_t d, int64_t t, double* X, int32_t* inv,
                       double* At, hipStream_t s) {
  if (r <= 0 || d <= 0 || t <= 0) return hipSuccess;
  int k = 0;
  while ((1ll << k) < r) ++k;
  const int h = std::max(1, (k + 1) / 2);
  fill_minus_one_kernel<<<(unsigned)((r + 255) / 256), 256, 0, s>>>(r, inv);
  srht_sample_kernel<<<(unsigned)((t + 255) / 256), 256, 0, s>>>(key_p, r, t, h, inv);
  const double scale = 1.0 / std::sqrt((double)t);
  const unsigned cblocks = (unsigned)((d + kCols - 1) / kCols);
  // passes of up to kMaxBits bits; at least one (r = 1 still applies D and P)
  int b0 = 0;
  do {
    const int nb = std::min(kMaxBits, k - b0);
    const bool first = b0 == 0, last = b0 + nb >= k;
    const dim3 grid((unsigned)(r >> nb), cblocks);
    fwht_pass_kernel<<<grid, kThreads, 0, s>>>(X, r, d, b0, nb, first, key_d, last, inv, scale, At);
    b0 += nb;
  } while (b0 < k);
  return hipGetLastError();
}

}  // namespace lev
