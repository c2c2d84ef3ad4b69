// Pass 2 for CSR input: theta~_i = || A[i, :] Z_full ||^2 (Algorithm 8, last
// step, on the selected columns; Z_full holds Z's rows at the selected
// columns' ids and zeros elsewhere).
//
// A sparse row times a dense d x k matrix has no dense tile for the matrix
// cores (a 16-row block of a 3%-dense A fills one 16x4 MFMA operand to a few
// percent), so this pass runs on the vector ALUs: every nonzero a_ij adds
// a_ij * Z_full[j, :] to the row's k-vector, one output column per lane.
// Z_full (padded to 64 columns) lives in LDS, shared by the 16 waves of a
// workgroup; each step gathers one 256-byte row of it, so the pass is bound
// by LDS bandwidth (about 256 B/clk per CU on gfx950) unless A's bytes are
// the larger cost.  Each wave streams a contiguous range of rows: the
// nonzeros of the range are read 64 at a time with coalesced loads and
// staged in a 64-entry LDS list (column offset into Z, value) that all lanes
// read by broadcast; row boundaries come from row_ptr and are uniform across
// the wave, so the step loop has no per-lane branches.  At a row boundary the
// squared k-vector is summed across the wave (DPP) into the row's lane of a
// result register, stored once per 64 rows.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kCsrWaves = 16;
constexpr int kCsrThreads = 64 * kCsrWaves;
constexpr int kZStride = 64;  // Z_full row stride in elements (k <= 64)
constexpr int kRowsPerTask = 64;

template <typename T>
__device__ __forceinline__ float to_f32(T x);
template <>
__device__ __forceinline__ float to_f32<float>(float x) { return x; }
template <>
__device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 x) {
  const uint16_t bits = *reinterpret_cast<const uint16_t*>(&x);
  return __uint_as_float((uint32_t)bits << 16);
}

// Sum over the 64 lanes (row shifts within 16-lane rows, then row
// broadcasts; lane 63 ends with the total), returned to every lane.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_sum_step(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v = dpp_sum_step<0x111, 0xF>(v);
  v = dpp_sum_step<0x112, 0xF>(v);
  v = dpp_sum_step<0x114, 0xF>(v);
  v = dpp_sum_step<0x118, 0xF>(v);
  v = dpp_sum_step<0x142, 0xA>(v);
  v = dpp_sum_step<0x143, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_sum_step(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return v + __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_sum_step<0x111, 0xF>(v);
  v = dpp_sum_step<0x112, 0xF>(v);
  v = dpp_sum_step<0x114, 0xF>(v);
  v = dpp_sum_step<0x118, 0xF>(v);
  v = dpp_sum_step<0x142, 0xA>(v);
  v = dpp_sum_step<0x143, 0xC>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t readlane64(int64_t x, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename ZT>
struct StageEntry {
  int off;   // element offset of Z_full's row in LDS (column id * kZStride)
  ZT val;
};

// G consecutive steps t .. t + G - 1 of the staged list: the G entry reads,
// then the G Z-row reads, then the products (alternating accumulators).
template <int G, typename ZT>
__device__ __forceinline__ void steps(const StageEntry<ZT>* my, const ZT* Z, int t, int lane, ZT& y, ZT& y2) {
  StageEntry<ZT> e[G];
  ZT z[G];
#pragma unroll
  for (int u = 0; u < G; ++u) e[u] = my[t + u];
#pragma unroll
  for (int u = 0; u < G; ++u) z[u] = Z[e[u].off + lane];
#pragma unroll
  for (int u = 0; u < G; u += 2) {
    y = fma(e[u].val, z[u], y);
    y2 = fma(e[u + 1].val, z[u + 1], y2);
  }
}

// T: storage type of A's values; ZT: type of Z_full and of the arithmetic
// (float for FP32/BF16 values, double for FP64 values).  ZLDS: Z_full staged
// in LDS (else read from global memory, for d * 64 * sizeof(ZT) beyond LDS).
template <typename T, typename ZT, bool ZLDS>
__global__ __launch_bounds__(kCsrThreads) void rownorm_csr_kernel(const T* __restrict__ vals,
                                                                  const int64_t* __restrict__ row_ptr,
                                                                  const int32_t* __restrict__ col_idx,
                                                                  int64_t n, int64_t d, int64_t nnz,
                                                                  const ZT* __restrict__ Zg,
                                                                  ZT* __restrict__ theta, ColTile ct) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (col_tile_dead(ct)) return;
  StageEntry<ZT>* stage = reinterpret_cast<StageEntry<ZT>*>(smem);  // [kCsrWaves][64]
  ZT* Zs = reinterpret_cast<ZT*>(smem + sizeof(StageEntry<ZT>) * 64 * kCsrWaves);
  const ZT* Z = ZLDS ? Zs : Zg;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (ZLDS) {
    const int64_t total = d * kZStride;
    for (int64_t e = threadIdx.x; e < total; e += kCsrThreads) Zs[e] = Zg[e];
    __syncthreads();
  }
  StageEntry<ZT>* my = stage + wave * 64;

  const int64_t ntask = (n + kRowsPerTask - 1) / kRowsPerTask;
  for (int64_t task = (int64_t)blockIdx.x * kCsrWaves + wave; task < ntask;
       task += (int64_t)gridDim.x * kCsrWaves) {
    const int64_t r0 = task * kRowsPerTask;
    const int64_t r1 = min(n, r0 + kRowsPerTask);
    // lane j holds row_ptr[r0 + j] (j <= r1 - r0; lane 64 would be r1 = r0 + 64)
    // Offsets are clamped to [0, nnz] and row ends to [pos, N1], so a
    // malformed row_ptr yields wrong rows but no stray access or endless loop.
    const int64_t rp = (r0 + lane <= r1) ? min(max(row_ptr[r0 + lane], (int64_t)0), nnz) : 0;
    const int64_t N0 = readlane64(rp, 0);
    const int64_t N1 = max(N0, min(max(row_ptr[r1], (int64_t)0), nnz));
    int64_t pos = N0;
    auto row_end = [&](int64_t row) -> int64_t {  // row_ptr[row + 1], row in [r0, r1)
      const int j = (int)(row + 1 - r0);
      return j < 64 ? min(max(readlane64(rp, j), pos), N1) : N1;
    };

    ZT out = 0;  // lane j: theta of row r0 + j
    ZT y = 0, y2 = 0;  // two accumulators: the unrolled steps alternate
    int64_t row = r0;
    int64_t rend = row_end(row);
    auto flush_rows = [&]() {
      while (row < r1 && rend == pos) {
        const ZT yy = y + y2;
        const ZT t = wave_sum(yy * yy);
        out = (lane == (int)(row - r0)) ? t : out;
        y = 0;
        y2 = 0;
        ++row;
        if (row < r1) rend = row_end(row);
      }
    };
    flush_rows();
    // the column ids and values of the next 64 nonzeros are loaded while the
    // current 64 are multiplied (one global round trip per chunk is no
    // longer on the wave's critical path)
    auto load_chunk = [&](int64_t cs, int32_t& c, T& v) {
      const int64_t p = cs + lane;
      const int64_t q = p < N1 ? p : (N1 > 0 ? N1 - 1 : 0);  // in bounds whenever nnz > 0
      c = p < N1 ? col_idx[q] : -1;
      v = p < N1 ? vals[q] : T{};
    };
    int32_t nc = -1;
    T nv{};
    if (N0 < N1) load_chunk(N0, nc, nv);
    for (int64_t c0 = N0; c0 < N1; c0 += 64) {
      const int32_t c = nc;
      const T cv = nv;
      if (c0 + 64 < N1) load_chunk(c0 + 64, nc, nv);
      StageEntry<ZT> e;
      e.off = 0;
      e.val = 0;
      if ((uint32_t)c < (uint32_t)d) {
        e.off = c * kZStride;
        if constexpr (sizeof(ZT) == 8) {
          e.val = (ZT)cv;
        } else {
          e.val = to_f32<T>(cv);
        }
      }
      my[lane] = e;
      __builtin_amdgcn_wave_barrier();
      const int64_t cend = min(c0 + 64, N1);
      while (pos < cend && row < r1) {
        const int stop = (int)(min(rend, cend) - c0);
        int t = (int)(pos - c0);
        // eight steps at a time: all sixteen LDS reads are issued before the
        // first product, so their latencies overlap; a segment's last steps
        // go in groups of 4, 2 and 1 (at most three dependent LDS round
        // trips instead of seven, and no step padded: with Z_full filling
        // LDS the pass runs four waves per SIMD and is bound by LDS issue
        // as much as by latency)
        for (; t + 8 <= stop; t += 8) steps<8>(my, Z, t, lane, y, y2);
        if (t + 4 <= stop) {
          steps<4>(my, Z, t, lane, y, y2);
          t += 4;
        }
        if (t + 2 <= stop) {
          steps<2>(my, Z, t, lane, y, y2);
          t += 2;
        }
        if (t < stop) {
          const StageEntry<ZT> e1 = my[t];
          y = fma(e1.val, Z[e1.off + lane], y);
        }
        pos = c0 + stop;
        flush_rows();
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (r0 + lane < r1) theta[r0 + lane] = ct.acc ? theta[r0 + lane] + out : out;
  }
}

template <typename T, typename ZT>
hipError_t launch_typed(const void* vals, const int64_t* row_ptr, const int32_t* col_idx, int64_t n, int64_t d,
                        int64_t nnz, const void* Zpack, void* theta, const ColTile& ct, hipStream_t s) {
  int dev = 0, num_cu = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  err = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (err != hipSuccess) return err;
  const size_t stage_bytes = sizeof(StageEntry<ZT>) * 64 * kCsrWaves;
  const size_t z_bytes = (size_t)d * kZStride * sizeof(ZT);
  constexpr size_t kMaxLds = 144 * 1024;  // leave room below the 160 KB of a CU
  const int64_t ntask = (n + kRowsPerTask - 1) / kRowsPerTask;
  const int64_t want = (ntask + kCsrWaves - 1) / kCsrWaves;
  const T* v = static_cast<const T*>(vals);
  const ZT* Z = static_cast<const ZT*>(Zpack);
  ZT* th = static_cast<ZT*>(theta);
  if (stage_bytes + z_bytes <= kMaxLds) {
    const size_t lds = stage_bytes + z_bytes;
    auto kern = rownorm_csr_kernel<T, ZT, true>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // one workgroup per CU holds the LDS copy of Z_full; a second fits when it is small
    const int per_cu = (2 * lds <= kMaxLds) ? 2 : 1;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * per_cu));
    kern<<<grid, kCsrThreads, lds, s>>>(v, row_ptr, col_idx, n, d, nnz, Z, th, ct);
  } else {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * 2));
    rownorm_csr_kernel<T, ZT, false><<<grid, kCsrThreads, stage_bytes, s>>>(v, row_ptr, col_idx, n, d, nnz, Z, th, ct);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rownorm_csr(int dtype, const void* vals, const int64_t* row_ptr, const int32_t* col_idx,
                              int64_t n, int64_t d, int64_t nnz, int64_t k, const void* Zpack,
                              const int64_t* live, void* theta, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int variant = dtype == 0 ? 6 : 5;
  // one pass per column tile of 64 (see launch_rownorm_dense)
  for (int64_t t = 0; t < z_tiles(k); ++t) {
    ColTile ct;
    ct.c0 = t * kZTile;
    ct.acc = t > 0;
    ct.live = t > 0 ? live : nullptr;
    const void* zt = static_cast<const char*>(Zpack) + pack_z_tile_offset(variant, d, k, t);
    hipError_t e = hipErrorInvalidValue;
    switch (dtype) {
      case 0: e = launch_typed<double, double>(vals, row_ptr, col_idx, n, d, nnz, zt, theta, ct, s); break;
      case 1: e = launch_typed<float, float>(vals, row_ptr, col_idx, n, d, nnz, zt, theta, ct, s); break;
      case 2: e = launch_typed<__hip_bfloat16, float>(vals, row_ptr, col_idx, n, d, nnz, zt, theta, ct, s); break;
      default: break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lev
