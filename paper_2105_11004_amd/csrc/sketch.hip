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
  const uint64_t x = hash_x(hp, (uint64_t)i);
  h_out[i] = (int64_t)((uint32_t)x % (uint32_t)hp.r_cs);  // x < P < 2^32
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

// Negates the elements of a 16-byte vector of T when neg is all ones (0:
// unchanged) by flipping their sign bits: exact, so adding the flipped
// value rounds exactly as adding s * x with s = -1 would.
template <typename T>
__device__ __forceinline__ void negate_if(uint4& raw, uint32_t neg);
template <>
__device__ __forceinline__ void negate_if<double>(uint4& raw, uint32_t neg) {
  raw.y ^= neg & 0x80000000u;
  raw.w ^= neg & 0x80000000u;
}
template <>
__device__ __forceinline__ void negate_if<float>(uint4& raw, uint32_t neg) {
  const uint32_t m = neg & 0x80000000u;
  raw.x ^= m;
  raw.y ^= m;
  raw.z ^= m;
  raw.w ^= m;
}
template <>
__device__ __forceinline__ void negate_if<__hip_bfloat16>(uint4& raw, uint32_t neg) {
  const uint32_t m = neg & 0x80008000u;
  raw.x ^= m;
  raw.y ^= m;
  raw.z ^= m;
  raw.w ^= m;
}

// Workgroup (blockIdx.x) share of the side draw: the pairs of the two
// matrices taken as one sequence, split over the first kDrawGroups
// workgroups (more when that would leave a thread over 16 pairs), one
// Box-Muller pair per thread and round.  Drawing in the workgroups that
// start first puts the matrices' stores ahead of most of the read stream
// (measured: 6-8 us less than spreading them over every workgroup).
constexpr int64_t kDrawGroups = 256;
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));
typedef float v2f_t __attribute__((ext_vector_type(2)));

// x = h + m + l exactly in FP32 for two values; BF16 parts packed in pairs
// (element 0 in the low half).
__device__ __forceinline__ void split3_pair(float x0, float x1, uint32_t& h, uint32_t& m, uint32_t& l) {
  auto pk = [](float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f_t){a, b}, v2bf_t));
  };
  h = pk(x0, x1);
  const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xFFFF0000u);
  m = pk(r0, r1);
  const float s0 = r0 - __uint_as_float(m << 16), s1 = r1 - __uint_as_float(m & 0xFFFF0000u);
  l = pk(s0, s1);
}

__device__ __forceinline__ void side_draw(const GaussDraw& g) {
  if (blockIdx.y != 0) return;
  const bool on0 = g.m[0].out != nullptr || g.m[0].parts3 != nullptr;
  const bool on1 = g.m[1].out != nullptr || g.m[1].parts3 != nullptr;
  const int64_t pairs0 = on0 ? (g.m[0].total + 1) / 2 : 0;
  const int64_t pairs1 = on1 ? (g.m[1].total + 1) / 2 : 0;
  const int64_t pairs = pairs0 + pairs1;
  if (pairs == 0) return;
  const int64_t want = max<int64_t>(kDrawGroups, (pairs + 16 * kThreads - 1) / (16 * kThreads));
  const int64_t groups = min<int64_t>((int64_t)gridDim.x, want);
  if ((int64_t)blockIdx.x >= groups) return;
  const int64_t per = (pairs + groups - 1) / groups;
  const int64_t q0 = (int64_t)blockIdx.x * per, q1 = min<int64_t>(q0 + per, pairs);
  for (int64_t qq = q0 + threadIdx.x; qq < q1; qq += blockDim.x) {
    const bool second = qq >= pairs0;
    const GaussMatrix& gm = second ? g.m[1] : g.m[0];
    const int64_t q = second ? qq - pairs0 : qq;
    double z0, z1;
    box_muller_pair((uint64_t)q, gm.key, &z0, &z1);
    // streaming stores: the matrix is read back only by the next kernel, and
    // non-temporal writes disturb pass 1's read stream less (measured ~3 us)
    if (gm.parts3 != nullptr) {
      // FP32 value split exactly into three BF16 parts (pairs packed)
      const float x0 = (float)(z0 * gm.scale);
      const float x1 = 2 * q + 1 < gm.total ? (float)(z1 * gm.scale) : 0.0f;
      uint32_t h, m, l;
      split3_pair(x0, x1, h, m, l);
      const int64_t np = (gm.total + 1) / 2;
      __builtin_nontemporal_store(h, gm.parts3 + q);
      __builtin_nontemporal_store(m, gm.parts3 + np + q);
      __builtin_nontemporal_store(l, gm.parts3 + 2 * np + q);
    } else {
      __builtin_nontemporal_store(z0 * gm.scale, gm.out + 2 * q);
      if (2 * q + 1 < gm.total) __builtin_nontemporal_store(z1 * gm.scale, gm.out + 2 * q + 1);
    }
  }
}

// One workgroup = one bucket x one column chunk of 64 * NV * E columns.
// Lane l of every wave covers 16-byte vectors v*64 + l (v < NV) of the
// chunk, so each wave reads NV contiguous KB-sized segments of a row.
// Wave w takes rows t = w, w + 4, ... of the staged row list, U at a time,
// with the next U rows in flight while the current ones are added.
template <typename T, int NV, int U, typename OutT>
__global__ __launch_bounds__(kThreads) void countsketch_dense_kernel(const T* __restrict__ A, int64_t d,
                                                                     int64_t ld, HashParams hp,
                                                                     OutT* __restrict__ SA, GaussDraw g) {
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
  side_draw(g);

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
    // The entries are the same for every lane: read as scalars, so the row
    // base is an SGPR pair and the sign a scalar mask that flips the sign
    // bits of the loaded row (rows past n load zeros and keep them).  Two
    // batches of U rows alternate, the next one in flight while the current
    // one is added.
    auto load_batch = [&](int q0, uint4 (&raw)[U][NV], uint32_t (&neg)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * kWaves;
        const uint32_t ent = __builtin_amdgcn_readfirstlane(q < cnt ? entries[q] : kInvalid);
        const bool ok = ent != kInvalid;
        neg[u] = (ok && (ent & 0x80000000u)) ? 0xFFFFFFFFu : 0u;
        const int64_t row = ok ? (int64_t)(ent & 0x7FFFFFFFu) : 0;
        const uint4* rp = reinterpret_cast<const uint4*>(A + row * ld + col0);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          raw[u][v] = (ok && vec_ok[v]) ? rp[v * 64 + lane] : make_uint4(0u, 0u, 0u, 0u);
      }
    };
    auto add_batch = [&](uint4 (&raw)[U][NV], const uint32_t (&neg)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          negate_if<T>(raw[u][v], neg[u]);
          double x[E];
          to_double<T>(raw[u][v], x);
#pragma unroll
          for (int e = 0; e < E; ++e) acc[v][e] += x[e];
        }
      }
    };
    uint4 ra[U][NV], rb[U][NV];
    uint32_t sa[U], sb[U];
    int q0 = wave;
    if (q0 < cnt) load_batch(q0, ra, sa);
    for (; q0 < cnt; q0 += 2 * kWaves * U) {
      const int q1 = q0 + kWaves * U;
      if (q1 < cnt) load_batch(q1, rb, sb);
      add_batch(ra, sa);
      if (q1 >= cnt) break;
      const int q2 = q1 + kWaves * U;
      if (q2 < cnt) load_batch(q2, ra, sa);
      add_batch(rb, sb);
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
      SA[b * d + col] = (OutT)s;
    }
  }
}

template <typename T, typename OutT>
hipError_t launch_dense_typed(const void* A, int64_t n, int64_t d, int64_t ld, const HashParams& hp,
                              OutT* SA, const GaussDraw& g, hipStream_t s) {
  (void)n;
  constexpr int E = Vec16<T>::E;
  const T* a = static_cast<const T*>(A);
  const int64_t per_vec_row = 64 * E;
  if (d <= per_vec_row) {
    dim3 grid((unsigned)hp.r_cs, 1);
    countsketch_dense_kernel<T, 1, 4, OutT><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA, g);
  } else if (d <= 2 * per_vec_row) {
    dim3 grid((unsigned)hp.r_cs, 1);
    countsketch_dense_kernel<T, 2, 2, OutT><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA, g);
  } else {
    const int64_t cols = 4 * per_vec_row;
    dim3 grid((unsigned)hp.r_cs, (unsigned)((d + cols - 1) / cols));
    countsketch_dense_kernel<T, 4, 1, OutT><<<grid, kThreads, 0, s>>>(a, d, ld, hp, SA, g);
  }
  return hipGetLastError();
}

// ---- CSR input -------------------------------------------------------------
// Same bucket-major gather as the dense kernel.  A wave takes the staged
// row list 64 entries at a time (lane j <-> entry j: its row's extent from
// row_ptr), then walks those rows U at a time: the first 64 nonzeros of U
// rows are loaded together (lane t <-> nonzero t of a row) and then added,
// row after row, into the wave's private FP64 accumulator in LDS with
// ds_add_f64.  Within one row the column ids are distinct, so one add
// instruction never hits an address twice, and the adds of one wave execute
// in program order: the accumulation order is a fixed function of the input
// and S A is bitwise reproducible.  The four wave accumulators are summed in
// a fixed order at the end.
template <typename T>
__device__ __forceinline__ double load_as_double(const T* p);
template <>
__device__ __forceinline__ double load_as_double<double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ double load_as_double<float>(const float* p) { return (double)*p; }
template <>
__device__ __forceinline__ double load_as_double<__hip_bfloat16>(const __hip_bfloat16* p) {
  const uint16_t bits = *reinterpret_cast<const uint16_t*>(p);
  return (double)__uint_as_float((uint32_t)bits << 16);
}

constexpr int kCsrU = 8;  // rows whose first 64 nonzeros are in flight together

template <typename T>
__global__ __launch_bounds__(kThreads) void countsketch_csr_kernel(const T* __restrict__ vals,
                                                                   const int64_t* __restrict__ row_ptr,
                                                                   const int32_t* __restrict__ col_idx,
                                                                   int64_t d, int64_t nnz, HashParams hp,
                                                                   double* __restrict__ SA, GaussDraw g) {
  extern __shared__ double acc[];  // [kWaves][d]
  __shared__ uint32_t entries[kChunk];
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* my = acc + (int64_t)wave * d;
  for (int64_t c = threadIdx.x; c < kWaves * d; c += kThreads) acc[c] = 0.0;
  side_draw(g);

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
    for (int q0 = wave * 64; q0 < cnt; q0 += kWaves * 64) {
      const int q = q0 + lane;
      const uint32_t ent = q < cnt ? entries[q] : kInvalid;
      int64_t start = 0;
      int len = 0;
      int neg = 0;
      if (ent != kInvalid) {
        const int64_t row = (int64_t)(ent & 0x7FFFFFFFu);
        // a well-formed row lies in [0, nnz) and has at most d nonzeros; the
        // clamps keep a malformed row_ptr from reading out of bounds
        start = min(max(row_ptr[row], (int64_t)0), nnz);
        const int64_t end = min(max(row_ptr[row + 1], start), nnz);
        len = (int)min<int64_t>(end - start, d);
        neg = (ent >> 31) != 0;
      }
      const int rows_here = min(64, cnt - q0);
      for (int g = 0; g < rows_here; g += kCsrU) {
        int32_t cv[kCsrU];
        double xv[kCsrU];
        int64_t st[kCsrU];
        int ln[kCsrU];
#pragma unroll
        for (int u = 0; u < kCsrU; ++u) {
          const int j = g + u;  // uniform
          const int jj = j < 64 ? j : 63;
          st[u] = ((int64_t)__builtin_amdgcn_readlane((int)(start >> 32), jj) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane((int)start, jj);
          ln[u] = j < rows_here ? __builtin_amdgcn_readlane(len, jj) : 0;
          const int sg = __builtin_amdgcn_readlane(neg, jj);
          cv[u] = 0;
          xv[u] = 0.0;
          if (lane < ln[u]) {
            cv[u] = col_idx[st[u] + lane];
            const double x = load_as_double<T>(vals + st[u] + lane);
            xv[u] = sg ? -x : x;
          }
        }
#pragma unroll
        for (int u = 0; u < kCsrU; ++u) {
          if (lane < ln[u] && (uint32_t)cv[u] < (uint32_t)d)
            __hip_atomic_fetch_add(my + cv[u], xv[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        // nonzeros beyond the first 64 of a row: row by row, up to 8 chunks
        // of 64 loaded together before they are added
#pragma unroll
        for (int u = 0; u < kCsrU; ++u) {
          const int sg = __builtin_amdgcn_readlane(neg, (g + u) < 64 ? g + u : 63);
          for (int off0 = 64; off0 < ln[u]; off0 += 8 * 64) {
            int32_t c8[8];
            double x8[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              const int off = off0 + 64 * v + lane;
              c8[v] = 0;
              x8[v] = 0.0;
              if (off < ln[u]) {
                c8[v] = col_idx[st[u] + off];
                const double x = load_as_double<T>(vals + st[u] + off);
                x8[v] = sg ? -x : x;
              }
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              if (off0 + 64 * v + lane < ln[u] && (uint32_t)c8[v] < (uint32_t)d)
                __hip_atomic_fetch_add(my + c8[v], x8[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  for (int64_t c = threadIdx.x; c < d; c += kThreads) {
    double s = acc[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += acc[(int64_t)w * d + c];
    SA[b * d + c] = s;
  }
}

template <typename T>
hipError_t launch_csr_typed(const void* vals, const int64_t* row_ptr, const int32_t* col_idx, int64_t d,
                            int64_t nnz, const HashParams& hp, double* SA, const GaussDraw& g, hipStream_t s) {
  const size_t lds = (size_t)kWaves * (size_t)d * sizeof(double);
  countsketch_csr_kernel<T><<<(unsigned)hp.r_cs, kThreads, lds, s>>>(static_cast<const T*>(vals), row_ptr,
                                                                      col_idx, d, nnz, hp, SA, g);
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
                                    const HashParams& hp, void* SA, bool sa_f32, const GaussDraw& g,
                                    hipStream_t s) {
  // FP32 S A only for BF16 input (the split-form transform's operand)
  if (sa_f32) {
    if (dtype != 2) return hipErrorInvalidValue;
    return launch_dense_typed<__hip_bfloat16>(A, n, d, ld, hp, static_cast<float*>(SA), g, s);
  }
  double* sa = static_cast<double*>(SA);
  switch (dtype) {
    case 0: return launch_dense_typed<double>(A, n, d, ld, hp, sa, g, s);
    case 1: return launch_dense_typed<float>(A, n, d, ld, hp, sa, g, s);
    case 2: return launch_dense_typed<__hip_bfloat16>(A, n, d, ld, hp, sa, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_countsketch_csr(int dtype, const void* vals, const int64_t* row_ptr, const int32_t* col_idx,
                                  int64_t n, int64_t d, int64_t nnz, const HashParams& hp, double* SA,
                                  const GaussDraw& g, hipStream_t s) {
  (void)n;
  switch (dtype) {
    case 0: return launch_csr_typed<double>(vals, row_ptr, col_idx, d, nnz, hp, SA, g, s);
    case 1: return launch_csr_typed<float>(vals, row_ptr, col_idx, d, nnz, hp, SA, g, s);
    case 2: return launch_csr_typed<__hip_bfloat16>(vals, row_ptr, col_idx, d, nnz, hp, SA, g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lev
