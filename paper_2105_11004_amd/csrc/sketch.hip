// Pass 1 of the estimator: the CountSketch product S A (Algorithm 3, first
// factor; CountSketch as defined in Section 3.4).
//
// Design.  S has one +-1 per column, so (S A)[b, :] = sum_{h(i) = b} s(i) A[i, :].
// Scatter-adding rows into S A with atomics would make the result depend on
// scheduling and costs one atomic per element.  Instead each workgroup owns
// one bucket b and gathers its rows.  The bucket hash is a permutation of
// [0, P) followed by "mod r_cs", so the rows of bucket b are the preimages of
// x = b, b + r_cs, b + 2 r_cs, ... < P, i.e. the arithmetic progression
// i_t = i_0 + t * delta (mod P) (rows >= n skipped).  No bucket structure is
// built or stored: pass 1 reads A exactly once and writes S A once, and the
// accumulation order (t ascending, fixed wave assignment, fixed cross-wave
// reduction) makes S A bitwise deterministic.  Accumulation is in FP64.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "lev_device.h"
#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 1024;              // row-list entries staged per step
constexpr uint32_t kInvalid = 0xFFFFFFFFu;  // sentinel (row ids < 2^31 - 1)

__global__ void hash_rows_kernel(HashParams hp, int64_t* h_out, int8_t* s_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hp.n) return;
  const uint64_t x = ((uint64_t)hp.a * (uint64_t)i + hp.c) % hp.P;
  h_out[i] = (int64_t)(x % (uint64_t)hp.r_cs);
  s_out[i] = sign_negative(hp, (uint64_t)i) ? (int8_t)-1 : (int8_t)1;
}

// Number of rows < n in each bucket's progression.
__global__ void bucket_count_kernel(HashParams hp, int64_t* cnt) {
  const int64_t b = blockIdx.x;
  const int64_t T = bucket_len(hp, b);
  const uint64_t i0 = T > 0 ? bucket_start(hp, b) : 0;
  int local = 0;
  for (int64_t t = threadIdx.x; t < T; t += blockDim.x)
    local += bucket_row(hp, i0, (uint64_t)t) < (uint64_t)hp.n;
  __shared__ int red[kThreads];
  red[threadIdx.x] = local;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[b + 1] = red[0];
}

// Exclusive scan of r_cs counts in place (off[0] = 0); one thread, debug only.
__global__ void serial_scan_kernel(int64_t* off, int64_t r_cs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  off[0] = 0;
  for (int64_t b = 0; b < r_cs; ++b) off[b + 1] += off[b];
}

// Writes bucket b's rows in progression order (one thread per bucket keeps
// the order trivially).
__global__ void bucket_fill_kernel(HashParams hp, const int64_t* off, int32_t* rows) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= hp.r_cs) return;
  const int64_t T = bucket_len(hp, b);
  const uint64_t i0 = T > 0 ? bucket_start(hp, b) : 0;
  int64_t pos = off[b];
  for (int64_t t = 0; t < T; ++t) {
    const uint64_t i = bucket_row(hp, i0, (uint64_t)t);
    if (i < (uint64_t)hp.n) rows[pos++] = (int32_t)i;
  }
}

template <typename T>
struct Vec16 {
  static constexpr int E = 16 / sizeof(T);
};

// Converts the 16-byte vector `raw` holding E elements of type T to double.
template <typename T>
__device__ __forceinline__ void to_double(const uint4& raw, double (&out)[Vec16<T>::E]);

template <>
__device__ __forceinline__ void to_double<double>(const uint4& raw, double (&out)[2]) {
  out[0] = __hiloint2double((int)raw.y, (int)raw.x);
  out[1] = __hiloint2double((int)raw.w, (int)raw.z);
}
template <>
__device__ __forceinline__ void to_double<float>(const uint4& raw, double (&out)[4]) {
  out[0] = (double)__uint_as_float(raw.x);
  out[1] = (double)__uint_as_float(raw.y);
  out[2] = (double)__uint_as_float(raw.z);
  out[3] = (double)__uint_as_float(raw.w);
}
template <>
__device__ __forceinline__ void to_double<__hip_bfloat16>(const uint4& raw, double (&out)[8]) {
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    out[2 * q] = (double)__uint_as_float(w[q] << 16);
    out[2 * q + 1] = (double)__uint_as_float(w[q] & 0xFFFF0000u);
  }
}

// One workgroup = one bucket x one column chunk of 64 * NV * E columns.
// Lane l of every wave covers 16-byte vectors v*64 + l (v < NV) of the
// chunk, so each wave reads NV contiguous KB-sized segments of a row.
// Wave w takes rows t = w, w + 4, ... of the staged row list, U at a time.
template <typename T, int NV, int U>
__global__ __launch_bounds__(kThreads) void countsketch_dense_kernel(const T* __restrict__ A, int64_t d,
                                                                     int64_t ld, HashParams hp,
                                                                     double* __restrict__ SA) {
  constexpr int E = Vec16<T>::E;
  constexpr int kCols = 64 * NV * E;
  __shared__ uint32_t entries[kChunk];
  __shared__ double red[kWaves][kCols];

  const int64_t b = blockIdx.x;
  const int64_t col0 = (int64_t)blockIdx.y * kCols;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;

  double acc[NV][E];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[v][e] = 0.0;

  bool vec_ok[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) vec_ok[v] = col0 + (int64_t)(v * 64 + lane) * E < d;

  const int64_t T_b = bucket_len(hp, b);
  const uint64_t i0 = T_b > 0 ? bucket_start(hp, b) : 0;

  for (int64_t t0 = 0; t0 < T_b; t0 += kChunk) {
    const int cnt = (int)min<int64_t>(kChunk, T_b - t0);
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += kThreads) {
      const uint64_t i = bucket_row(hp, i0, (uint64_t)(t0 + q));
      uint32_t e = kInvalid;
      if (i < (uint64_t)hp.n) e = (uint32_t)i | (sign_negative(hp, i) ? 0x80000000u : 0u);
      entries[q] = e;
    }
    __syncthreads();
    for (int q0 = wave; q0 < cnt; q0 += kWaves * U) {
      uint4 raw[U][NV];
      double sgn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * kWaves;
        const uint32_t ent = q < cnt ? entries[q] : kInvalid;
        const bool ok = ent != kInvalid;
        sgn[u] = ok ? ((ent & 0x80000000u) ? -1.0 : 1.0) : 0.0;
        const int64_t row = ok ? (int64_t)(ent & 0x7FFFFFFFu) : 0;
        const uint4* rp = reinterpret_cast<const uint4*>(A + row * ld + col0);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          raw[u][v] = (ok && vec_ok[v]) ? rp[v * 64 + lane] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double x[E];
          to_double<T>(raw[u][v], x);
#pragma unroll
          for (int e = 0; e < E; ++e) acc[v][e] = fma(sgn[u], x[e], acc[v][e]);
        }
      }
    }
  }

#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < E; ++e) red[wave][(v * 64 + lane) * E + e] = acc[v][e];
  __syncthreads();
  for (int cidx = threadIdx.x; cidx < kCols; cidx += kThreads) {
    const int64_t col = col0 + cidx;
    if (col < d) {
      double s = red[0][cidx];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) s += red[w][cidx];
      SA[b * d + col] = s;
    }
  }
}

template <typename T>
hipError_t launch_dense_typed(const void* A, int64_t n, int64_t d, int64_t ld, const HashParams& hp,
                              double* SA, hipStream_t s) {
  (void)n;
  constexpr int E = Vec16<T>::E;
  const T* a = static_cast<const T*>(A);
  const int64_t per_vec_row = 64 * E;
  if (d <= per_vec_row) {
    dim3 grid((unsigned)hp.r_cs, 1);
    countsketch_dense_kernel<T, 1, 8><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA);
  } else if (d <= 2 * per_vec_row) {
    dim3 grid((unsigned)hp.r_cs, 1);
    countsketch_dense_kernel<T, 2, 4><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA);
  } else {
    const int64_t cols = 4 * per_vec_row;
    dim3 grid((unsigned)hp.r_cs, (unsigned)((d + cols - 1) / cols));
    countsketch_dense_kernel<T, 4, 2><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_hash_rows(const HashParams& hp, int64_t* h_out, int8_t* s_out, hipStream_t s) {
  if (hp.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((hp.n + 255) / 256);
  hash_rows_kernel<<<blocks, 256, 0, s>>>(hp, h_out, s_out);
  return hipGetLastError();
}

hipError_t launch_bucket_lists(const HashParams& hp, int64_t* off, int32_t* rows, hipStream_t s) {
  hipError_t e = launch_fill_zero(off, sizeof(int64_t) * (size_t)(hp.r_cs + 1), s);
  if (e != hipSuccess) return e;
  bucket_count_kernel<<<(unsigned)hp.r_cs, kThreads, 0, s>>>(hp, off);
  serial_scan_kernel<<<1, 64, 0, s>>>(off, hp.r_cs);
  bucket_fill_kernel<<<(unsigned)((hp.r_cs + 255) / 256), 256, 0, s>>>(hp, off, rows);
  return hipGetLastError();
}

hipError_t launch_countsketch_dense(int dtype, const void* A, int64_t n, int64_t d, int64_t ld,
                                    const HashParams& hp, double* SA, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_dense_typed<double>(A, n, d, ld, hp, SA, s);
    case 1: return launch_dense_typed<float>(A, n, d, ld, hp, SA, s);
    case 2: return launch_dense_typed<__hip_bfloat16>(A, n, d, ld, hp, SA, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lev
