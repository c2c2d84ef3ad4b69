// Pass 2 for A stored in BF16 (Algorithm 8, last step, on the selected
// columns): theta~_i = || A[i, :] Z_full ||^2 on the BF16 matrix cores, with
// Z_full held as NP BF16 parts (1: Z rounded to BF16; 2: hi + lo; 3: hi +
// mid + lo, which carries Z to ~2^-27 so that, A being exact in BF16, every
// product is as accurate as an FP32 product and the pass matches the FP32
// estimator).
//
// Why a separate kernel.  With three parts Z_full is 3 * d * 64 * 2 bytes
// (384 KB at d = 1024): more than a CU's LDS, and a wave that owns 16 rows
// would re-read all of it per 16 rows (12 bytes of Z per byte of A).  Here
// a workgroup of 8 waves walks the contraction in chunks of 32 columns, with
// Z staged through LDS a few chunks at a time, and each wave owns 64 rows
// (four 16-row MFMA tiles), so every Z fragment read from LDS feeds four
// products: per chunk a workgroup reads 32 KB of A from HBM and NP * CB *
// 8 KB of Z from LDS, and runs 32 * NP * CB MFMAs.  (Measured: with two
// tiles per wave the LDS reads of Z, not the matrix cores, were what the
// pass waited on.)
//
// Pipeline.  The workgroup's work is a sequence of steps g, one per (row
// block, chunk) pair, grouped in windows of kW = 4 steps.  The A fragments of
// step g + P are loaded into a register ring P steps ahead (no branch around
// a load, so they stay in flight across steps).  Z lives in LDS as two
// windows of kW chunks: window w is read from slot group w & 1; at its start
// the chunks of window w + 1 (loaded into registers during window w - 1)
// are written into the other group and those of window w + 2 are loaded;
// one barrier per window.  Group (w + 1) & 1 was last read in window w - 1,
// which every wave finished before the barrier that opened window w.
// Between barriers the waves run freely, so one wave's LDS reads overlap
// another's matrix-core work.
//
// Accuracy: products are exact in FP32 (BF16 x BF16) and the matrix cores
// accumulate each output y_ic over the row in FP32, as an FP32 GEMM does
// (relative error about u_32 sqrt(d / 32) for sums without cancellation);
// the squares and their sum over the k columns are taken in FP64.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kTiles = 4;                            // 16-row MFMA tiles per wave
constexpr int kRowsPerWave = 16 * kTiles;
constexpr int kBlockRows = kWaves * kRowsPerWave;    // 512 rows per row block
constexpr int kW = 4;                                // steps per window (per barrier)
constexpr int kP = kW;                               // A: steps in flight per thread

__device__ __forceinline__ v8bf as_bf(const uint4& u) { return __builtin_bit_cast(v8bf, u); }

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// waits for every outstanding global load, which would drain the prefetch
// ring at every chunk; here the only data exchanged between waves is the Z
// chunk in LDS.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <typename T>
__device__ __forceinline__ T sum16(T x) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Z chunk layout (packed by trsm.hip, variants 2/3/4): part p, vector
// (t * CB + cb) * 64 + lane at Zg[p * part_vecs + (t * CB + cb) * 64 + lane];
// value = Z_full[32 t + 8 (lane / 16) + e][16 cb + lane % 16], e < 8.  In
// LDS a chunk is [p][cb][lane] (Q = NP * CB * 64 vectors) and a window kW
// chunks; thread i stages vectors i, i + kThreads, ... of a window.
template <int NP, int CB>
struct ZChunk {
  static constexpr int Q = NP * CB * 64;
  static constexpr int kWin = kW * Q;                              // vectors per window
  static constexpr int kPer = (kWin + kThreads - 1) / kThreads;    // per thread
};

template <int NP, int CB>
__global__ __launch_bounds__(kThreads, 1) void rownorm_bf16s_kernel(
    const __hip_bfloat16* __restrict__ A, int64_t n, int64_t d, int64_t ld, int nt, const uint4* __restrict__ Zg,
    int64_t part_vecs, float* __restrict__ theta, int64_t nblocks, ColTile ct) {
  using ZC = ZChunk<NP, CB>;
  __shared__ uint4 zs[2][ZC::kWin];
  if (col_tile_dead(ct)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g4 = lane >> 4;
  const bool whole_d = (d % 32) == 0;
  const bool theta_vec = (reinterpret_cast<uintptr_t>(theta) & 15) == 0;

  // the workgroup's row blocks: blockIdx.x, blockIdx.x + gridDim.x, ...
  const int64_t my_blocks = nblocks > blockIdx.x ? (nblocks - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t total = my_blocks * nt;  // chunk steps
  if (total == 0) return;

  // A cursor over the workgroup's steps: (row block, chunk) advanced one
  // step at a time (no divisions), with the lane's row pointers of the two
  // tiles.  Rows past n read row 0 (their results are never stored).
  struct Cursor {
    int64_t blk;  // row block index
    int t;        // chunk
  };
  const int64_t lane_row = (int64_t)wave * kRowsPerWave + (lane & 15);
  auto row_ptr = [&](int64_t blk, int h) -> const __hip_bfloat16* {
    const int64_t row = blk * kBlockRows + lane_row + 16 * h;
    return A + (row < n ? row : 0) * ld;
  };
  auto advance = [&](Cursor& c) {
    if (++c.t == nt) {
      c.t = 0;
      c.blk += gridDim.x;
    }
  };
  // A fragment of tile h at chunk t: lane's 8 BF16 at columns 32 t + 8 (lane
  // / 16) ... .  Columns past d (the ragged last chunk, where col + 8 <= ld
  // still holds since ld is a multiple of 8) are read as they are and zeroed
  // by mask_a when the fragment is used: no branch around a load, so the
  // loads stay in flight across the steps.
  auto load_a = [&](const __hip_bfloat16* rp, int t) -> uint4 {
    const int col = t * 32 + 8 * g4;
    return *reinterpret_cast<const uint4*>(rp + (col < d ? col : 0));
  };
  auto mask_a = [&](uint4 v, int t) -> uint4 {
    const int col = t * 32 + 8 * g4;
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t m = (col + 2 * i < d ? 0x0000FFFFu : 0u) | (col + 2 * i + 1 < d ? 0xFFFF0000u : 0u);
      w[i] &= m;
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  };
  // this thread's Z vectors of the window whose first step is at chunk t0:
  // vector q = tid + j * kThreads is part p, column block and lane rem of the
  // window's chunk c = q / Q, i.e. chunk (t0 + c) mod nt of the sequence
  // (vector j of this thread, one value per call: passing the staging array
  // by reference lets the compiler move it to LDS)
  // (the part of the index that depends on the thread and j only is
  // computed once: zk[j] = (p * part_vecs + rem) * 4 + c, c < kW = 4)
  static_assert(kW <= 4, "the chunk of a window is kept in two bits of zk");
  int zk[ZC::kPer];
#pragma unroll
  for (int j = 0; j < ZC::kPer; ++j) {
    int q = tid + j * kThreads;
    if (q >= ZC::kWin) q = ZC::kWin - 1;  // (duplicate of a valid vector, not stored)
    const int c = q / ZC::Q, qq = q % ZC::Q;
    const int p = qq / (CB * 64), rem = qq % (CB * 64);
    zk[j] = (int)(p * part_vecs + rem) * 4 + c;
  }
  auto load_zvec = [&](int t0, int j) -> uint4 {
    // chunk c of the window, wrapped at nt
    int t = t0 + (zk[j] & 3);
    t = t >= nt ? t - nt : t;
    t = t >= nt ? t - nt : t;
    t = t >= nt ? t - nt : t;
    return Zg[(zk[j] >> 2) + t * (CB * 64)];
  };
#define LEV_LOAD_ZWIN(T0)                                                  \
  _Pragma("unroll") for (int j = 0; j < ZC::kPer; ++j) zstage[j] = load_zvec((T0), j);
#define LEV_STORE_ZWIN(GRP)                                                \
  _Pragma("unroll") for (int j = 0; j < ZC::kPer; ++j) {                   \
    const int q = tid + j * kThreads;                                      \
    if (q < ZC::kWin) zs[(GRP)][q] = zstage[j];                            \
  }

  uint4 aring[kP][kTiles];
  uint4 zstage[ZC::kPer];
  // prologue: A of steps 0 .. P-1 in flight (clamped to the last step),
  // window 0's Z into group 0, window 1's Z into registers; pre = the step
  // the next A refill loads
  const int wstep = kW % nt;
  auto next_t = [&](int t) { return t + wstep >= nt ? t + wstep - nt : t + wstep; };
  Cursor cur{(int64_t)blockIdx.x, 0};
  Cursor pre = cur;
  int64_t pre_g = 0;
  // the refill cursor's row pointers, recomputed only when it moves to the
  // next row block (every nt steps), not at every step
  const __hip_bfloat16* prp[kTiles];
#pragma unroll
  for (int h = 0; h < kTiles; ++h) prp[h] = row_ptr(pre.blk, h);
  auto advance_pre = [&]() {
    if (pre_g + 1 < total) {
      ++pre_g;
      if (++pre.t == nt) {
        pre.t = 0;
        pre.blk += gridDim.x;
#pragma unroll
        for (int h = 0; h < kTiles; ++h) prp[h] = row_ptr(pre.blk, h);
      }
    }
  };
  LEV_LOAD_ZWIN(0)
#pragma unroll
  for (int u = 0; u < kP; ++u) {
#pragma unroll
    for (int h = 0; h < kTiles; ++h) aring[u][h] = load_a(prp[h], pre.t);
    advance_pre();
  }
  LEV_STORE_ZWIN(0)
  int zt = next_t(0);  // first chunk of window 1
  LEV_LOAD_ZWIN(zt)
  zt = next_t(zt);
  lds_barrier();

  v4f acc[kTiles][CB];
#pragma unroll
  for (int h = 0; h < kTiles; ++h)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[h][cb] = v4f{0.f, 0.f, 0.f, 0.f};

  // steps past total (up to two whole windows) are dummies: they load the
  // last step again, multiply into accumulators that are never stored, and
  // keep the barriers in step.  Two windows per iteration, so the ring slot
  // u % kP and the LDS group (u / kW) are compile-time constants.
  const int64_t steps = (total + 2 * kW - 1) / (2 * kW) * (2 * kW);
  for (int64_t g0 = 0; g0 < steps; g0 += 2 * kW) {
#pragma unroll
    for (int u = 0; u < 2 * kW; ++u) {
      const int slot = u % kP;
      const int grp = u / kW;
      if (u % kW == 0) {
        // window start: the next window's Z (loaded during the previous
        // window) into the other group, last read in the previous window;
        // then the window after next into registers
        LEV_STORE_ZWIN(grp ^ 1)
        LEV_LOAD_ZWIN(zt)
        zt = next_t(zt);
      }
      const int64_t g = g0 + u;
      const bool real = g < total;  // uniform across the workgroup
      const int t = cur.t;
      // the step's operands (ring slot u); the slot is refilled with step pre
      // (g + P, clamped to the last step) once the MFMAs have read it, so no
      // copy of a value still in flight is needed
      // (one uniform branch around all the masking, so that its arithmetic
      // is not hoisted into the steps of whole chunks)
      uint4 a[kTiles];
#pragma unroll
      for (int h = 0; h < kTiles; ++h) a[h] = aring[slot][h];
      if (!whole_d) {
#pragma unroll
        for (int h = 0; h < kTiles; ++h) a[h] = mask_a(a[h], t);
      }
      // chunk t: lo parts first (smallest terms first)
      const uint4* zb = zs[grp] + (u % kW) * ZC::Q;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        uint4 z[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) z[p] = zb[(p * CB + cb) * 64 + lane];
#pragma unroll
        for (int p = NP - 1; p >= 0; --p)
#pragma unroll
          for (int h = 0; h < kTiles; ++h)
            acc[h][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[h]), as_bf(z[p]), acc[h][cb], 0, 0, 0);
      }
#pragma unroll
      for (int h = 0; h < kTiles; ++h) aring[slot][h] = load_a(prp[h], pre.t);
      advance_pre();
      if (t == nt - 1) {
        // theta of the wave's rows: accumulator element v of lane l is row
        // 4 (l / 16) + v of its tile, column 16 cb + l % 16
        const int64_t row0 = cur.blk * kBlockRows + wave * kRowsPerWave;
#pragma unroll
        for (int h = 0; h < kTiles; ++h) {
          double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const double y = (double)acc[h][cb][v];
              sq[v] = fma(y, y, sq[v]);
            }
            acc[h][cb] = v4f{0.f, 0.f, 0.f, 0.f};
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) sq[v] = sum16(sq[v]);
          if (real && (lane & 15) == 0) {
            const int64_t r0 = row0 + 16 * h + 4 * g4;
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
      advance(cur);
      if (u % kW == kW - 1) lds_barrier();
    }
  }
#undef LEV_LOAD_ZWIN
#undef LEV_STORE_ZWIN
}

template <int NP, int CB>
hipError_t launch_np_cb(const __hip_bfloat16* A, int64_t n, int64_t d, int64_t ld, int nt, const uint4* Z,
                        int64_t part_vecs, float* theta, const ColTile& ct, hipStream_t s) {
  int dev = 0, num_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t nblocks = (n + kBlockRows - 1) / kBlockRows;
  // one workgroup per CU (its 8 waves take half of each SIMD's registers),
  // persistent over the row blocks
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nblocks, num_cu));
  rownorm_bf16s_kernel<NP, CB><<<(unsigned)grid, kThreads, 0, s>>>(A, n, d, ld, nt, Z, part_vecs, theta, nblocks, ct);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_np(const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* Zpack, void* theta,
                     const ColTile& ct, hipStream_t s) {
  const int nt = (int)((d + 31) / 32);
  const int64_t cbn = (k + 15) / 16;
  const int64_t part_vecs = (int64_t)nt * cbn * 64;
  const auto* a = static_cast<const __hip_bfloat16*>(A);
  const auto* z = static_cast<const uint4*>(Zpack);
  auto* th = static_cast<float*>(theta);
  switch (cbn) {
    case 1: return launch_np_cb<NP, 1>(a, n, d, ld, nt, z, part_vecs, th, ct, s);
    case 2: return launch_np_cb<NP, 2>(a, n, d, ld, nt, z, part_vecs, th, ct, s);
    case 3: return launch_np_cb<NP, 3>(a, n, d, ld, nt, z, part_vecs, th, ct, s);
    case 4: return launch_np_cb<NP, 4>(a, n, d, ld, nt, z, part_vecs, th, ct, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_rownorm_bf16(int parts, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k,
                               const void* Zpack, void* theta, const ColTile& ct, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (parts) {
    case 1: return launch_np<1>(A, n, d, ld, k, Zpack, theta, ct, s);
    case 2: return launch_np<2>(A, n, d, ld, k, Zpack, theta, ct, s);
    case 3: return launch_np<3>(A, n, d, ld, k, Zpack, theta, ct, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lev
