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
// (with every row on, a lane whose source is outside its row reads 0 either
// way; bound_ctrl says so, so no zeroed copy of the old value is made)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_sum_step(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, ROWMASK == 0xF));
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
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, ROWMASK == 0xF);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, ROWMASK == 0xF);
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

// ---- FP32 Z: rows shared out to 16-lane groups --------------------------------
// A wave takes 64 consecutive rows.  Lane l of group g (16 lanes) owns
// columns 4 (l % 16) .. + 3 of the k <= 64 output columns, and a group walks
// one row's nonzeros 16 at a time: each lane loads one (column id, value),
// then for each of the 16 entries the group broadcasts it from its lane (DPP
// row_newbcast, no LDS), reads the 16 bytes of Z_full's row it needs
// (ds_read_b128: the group reads the whole 256-byte row, conflict-free) and
// does four FMAs.  A row of at most one nonzero a_ij needs no k-vector:
// theta = a_ij^2 ||Z_full[j,:]||^2, from the squared row norms of Z_full
// kept in LDS beside it, one row a lane.  The other light rows (2 .. 63
// nonzeros) go four at a time, one per group.  The four groups move in step, so a wave pays for the longest of
// its four rows: the light rows of the 64 are first ordered by length class
// (1, 2, 3-4, 5-8, ..., 33-63; counted with ballots, moved with a forward
// lane permutation), which puts rows of similar length side by side (with
// power-law row lengths, a third of the group steps did useful work in row
// order).  Short chunks step one entry at a time up to four, then four at a
// time.  Heavy rows are split over the four groups, entry c0 + 4 i + g of
// a 64-entry chunk going to lane i of group g, so a chunk's last partial
// stretch costs a quarter of its length, and the groups' partial k-vectors
// are added at the end.
// Z_full sits in LDS unpadded, 256 bytes a row: a group's 16-lane read is
// one whole row (measured on gfx950: a 68-float stride cost two bank-
// conflict cycles per LDS instruction, 64 none).  The squares of a row's k-vector
// are summed over the group with four DPP steps; the group's last lane
// stores theta.
constexpr int kGZStride = 64;
constexpr int kHeavy = 64;

template <int U>
__device__ __forceinline__ int row_bcast_i(int v) {
  // every lane reads a valid lane of its row and all rows and banks are on, so
  // the old value is never used (bound_ctrl set: no copy of it is made)
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + U, 0xF, 0xF, true);  // row_newbcast:U
}

__device__ __forceinline__ float group_sum16(float v) {
  // prefix within each 16-lane row; lane 15 of the row ends with the total
  v = dpp_sum_step<0x111, 0xF>(v);
  v = dpp_sum_step<0x112, 0xF>(v);
  v = dpp_sum_step<0x114, 0xF>(v);
  v = dpp_sum_step<0x118, 0xF>(v);
  return v;
}

// y += the group's first `steps` (wave-uniform; rounded up to 4 past 4, at
// most 16) staged entries (col, val); masked entries carry a zero value.
__device__ __forceinline__ void group_chunk(const float* __restrict__ Zs, int col, float val, int gl, float (&y)[4],
                                            int steps = 16) {
#define LEV_GSTEP(U)                                                                                   \
  {                                                                                                  \
    const int cu = row_bcast_i<U>(col);                                                              \
    const float vu = __int_as_float(row_bcast_i<U>(__float_as_int(val)));                            \
    const float4 z = *reinterpret_cast<const float4*>(Zs + cu * kGZStride + 4 * gl);                 \
    y[0] = fmaf(vu, z.x, y[0]);                                                                      \
    y[1] = fmaf(vu, z.y, y[1]);                                                                      \
    y[2] = fmaf(vu, z.z, y[2]);                                                                      \
    y[3] = fmaf(vu, z.w, y[3]);                                                                      \
  }
  LEV_GSTEP(0)
  if (steps > 1) LEV_GSTEP(1)
  if (steps > 2) LEV_GSTEP(2)
  if (steps > 3) LEV_GSTEP(3)
  if (steps > 4) { LEV_GSTEP(4) LEV_GSTEP(5) LEV_GSTEP(6) LEV_GSTEP(7) }
  if (steps > 8) { LEV_GSTEP(8) LEV_GSTEP(9) LEV_GSTEP(10) LEV_GSTEP(11) }
  if (steps > 12) { LEV_GSTEP(12) LEV_GSTEP(13) LEV_GSTEP(14) LEV_GSTEP(15) }
#undef LEV_GSTEP
}

template <typename T>
__global__ __launch_bounds__(kCsrThreads) void rownorm_csr_grp_kernel(const T* __restrict__ vals,
                                                                      const int64_t* __restrict__ row_ptr,
                                                                      const int32_t* __restrict__ col_idx,
                                                                      int64_t n, int64_t d, int64_t nnz,
                                                                      const float* __restrict__ Zg,
                                                                      float* __restrict__ theta, ColTile ct) {
  extern __shared__ __align__(16) float Zs[];  // d rows of kGZStride floats, then d squared row norms
  if (col_tile_dead(ct)) return;
  float* zn = Zs + d * kGZStride;
  for (int64_t e = threadIdx.x; e < d * 64; e += kCsrThreads) Zs[(e / 64) * kGZStride + (e % 64)] = Zg[e];
  for (int64_t c = threadIdx.x; c < d; c += kCsrThreads) {
    float a = 0.f;
    for (int q = 0; q < 64; ++q) a = fmaf(Zg[c * 64 + q], Zg[c * 64 + q], a);
    zn[c] = a;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4, gl = lane & 15;
  const int64_t ntask = (n + 63) / 64;
  const int64_t tstep = (int64_t)gridDim.x * kCsrWaves;
  int64_t task = (int64_t)blockIdx.x * kCsrWaves + wave;
  // the next task's row starts load while the current task runs
  auto row_start = [&](int64_t tk) -> int64_t {
    if (tk >= ntask) return 0;
    const int64_t r = tk * 64 + lane;
    return r <= n ? min(max(row_ptr[r], (int64_t)0), nnz) : nnz;
  };
  int64_t rp_next = row_start(task);
  for (; task < ntask; task += tstep) {
    const int64_t r0 = task * 64;
    const int nr = (int)min((int64_t)64, n - r0);
    // lane j: start of row r0 + j, made non-decreasing
    int64_t rp = rp_next;
    rp_next = row_start(task + tstep);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t up = __shfl_up(rp, o, 64);
      if (lane >= o) rp = max(rp, up);
    }
    int64_t last = min(max(row_ptr[r0 + nr], (int64_t)0), nnz);
    last = max(last, __shfl(rp, 63, 64));
    if (lane >= nr) rp = last;  // rows past the task's end are empty
    // (the shuffle runs on every lane: a lane masked off by a branch does not
    // supply its value to the others)
    const int64_t down = __shfl_down(rp, 1, 64);
    const int64_t rnext = lane < 63 ? down : last;
    const int len = lane < nr ? (int)(rnext - rp) : 0;
    const uint64_t heavy = __ballot(lane < nr && len >= kHeavy);
    // rows of at most one nonzero, one a lane (an empty row's theta is 0)
    if (lane < nr && len <= 1) {
      float sq = 0.f;
      if (len == 1) {
        const int cc = col_idx[rp];
        const float vv = to_f32<T>(vals[rp]);
        if ((uint32_t)cc < (uint32_t)d) sq = vv * vv * zn[cc];
      }
      const int64_t r = r0 + lane;
      theta[r] = ct.acc ? theta[r] + sq : sq;
    }
    // the other light rows by length class; sorted position q holds row
    // srow, its start rps and length lens; the rows just done (class 0),
    // then the heavy rows and lanes past the task's end sort outside
    // positions n01 .. nlight - 1
    const bool light = lane < nr && len < kHeavy;
    const int cls = light ? (len <= 1 ? 0 : 32 - __builtin_clz((unsigned)(len - 1))) : 7;
    int pos = 0, base = 0, nlight = 0, n01 = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint64_t m = __ballot(cls == c);
      const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (cls == c) pos = base + below;
      base += __popcll(m);
      if (c == 0) n01 = base;
      if (c == 6) nlight = base;
    }
    const int srow = __builtin_amdgcn_ds_permute(4 * pos, lane);
    const int64_t rps = ((int64_t)__builtin_amdgcn_ds_permute(4 * pos, (int)(rp >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_ds_permute(4 * pos, (int)rp);
    const int lens = __builtin_amdgcn_ds_permute(4 * pos, light ? len : 0);

    // light rows of 2 .. 63 nonzeros: group g takes sorted positions
    // n01 + 4 q + g; the first 32 nonzeros of the rows two steps ahead load
    // while a step runs (a ring of three); a position at or past nlight
    // (possibly past the wave) stands for an empty row
    int pc[3][2];
    float pv[3][2];
#define LEV_LOADQ(Q, SLOT)                                                                          \
    {                                                                                               \
      const int jj = n01 + 4 * (Q) + g;                                                             \
      const int64_t ss = __shfl(rps, jj & 63, 64);                                                  \
      const int lr = __shfl(lens, jj & 63, 64); /* on every lane, then masked */                    \
      const int ll = jj < nlight ? lr : 0;                                                          \
      _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                               \
        const int t = 16 * h + gl;                                                                  \
        const bool ok = t < ll;                                                                     \
        const int cc = ok ? col_idx[ss + t] : 0;                                                    \
        const float vv = ok ? to_f32<T>(vals[ss + t]) : 0.f;                                        \
        const bool cin = (uint32_t)cc < (uint32_t)d;                                                \
        pc[SLOT][h] = cin ? cc : 0;                                                                 \
        pv[SLOT][h] = cin ? vv : 0.f;                                                               \
      }                                                                                             \
    }
    LEV_LOADQ(0, 0)
    LEV_LOADQ(1, 1)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (n01 + 4 * q >= nlight) break;  // uniform: the rest are heavy or past the end
      if (q + 2 < 16) LEV_LOADQ(q + 2, (q + 2) % 3)
      const int slot = q % 3;
      const int j = n01 + 4 * q + g;
      const bool mine = j < nlight;
      const int64_t s0 = __shfl(rps, j & 63, 64);
      const int ljr = __shfl(lens, j & 63, 64);  // on every lane, then masked
      const int lj = mine ? ljr : 0;
      // wave-uniform chunk count: the longest of the four groups' rows
      int mx = lj;
      mx = max(mx, __shfl_xor(mx, 16, 64));
      mx = max(mx, __shfl_xor(mx, 32, 64));
      float y[4] = {0.f, 0.f, 0.f, 0.f};
      if (mx > 0) group_chunk(Zs, pc[slot][0], pv[slot][0], gl, y, mx);
      if (mx > 16) group_chunk(Zs, pc[slot][1], pv[slot][1], gl, y, mx - 16);
      for (int c0 = 32; c0 < mx; c0 += 16) {
        const int t = c0 + gl;
        const bool ok = t < lj;
        const int col = ok ? col_idx[s0 + t] : 0;
        const float v = ok ? to_f32<T>(vals[s0 + t]) : 0.f;
        const bool cin = (uint32_t)col < (uint32_t)d;
        group_chunk(Zs, cin ? col : 0, cin ? v : 0.f, gl, y, mx - c0);
      }
      const float sq = group_sum16(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
      const int sj = __shfl(srow, j & 63, 64);
      if (mine && gl == 15) {
        const int64_t r = r0 + sj;
        theta[r] = ct.acc ? theta[r] + sq : sq;
      }
    }
#undef LEV_LOADQ
    // heavy rows: the four groups split each row's nonzeros (entry c0 + 4 i
    // + g to lane i of group g); the next chunk of 64 loads while the
    // current one runs
    uint64_t hm = heavy;
    while (hm) {
      const int j = __builtin_ctzll(hm);
      hm &= hm - 1;
      const int64_t s0 = __shfl(rp, j, 64);
      const int lj = __shfl(len, j, 64);
      auto load = [&](int c0, int& col, float& v) {
        const int t = c0 + 4 * gl + g;
        const bool ok = t < lj;
        const int cc = ok ? col_idx[s0 + t] : 0;
        const float vv = ok ? to_f32<T>(vals[s0 + t]) : 0.f;
        const bool cin = (uint32_t)cc < (uint32_t)d;
        col = cin ? cc : 0;
        v = cin ? vv : 0.f;
      };
      int col;
      float v;
      load(0, col, v);
      float y[4] = {0.f, 0.f, 0.f, 0.f};
      for (int c0 = 0; c0 < lj; c0 += 64) {
        int ncol = 0;
        float nv = 0.f;
        if (c0 + 64 < lj) load(c0 + 64, ncol, nv);
        group_chunk(Zs, col, v, gl, y, min(16, (lj - c0 + 3) / 4));
        col = ncol;
        v = nv;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        y[q] += __shfl_xor(y[q], 16, 64);
        y[q] += __shfl_xor(y[q], 32, 64);
      }
      const float sq = group_sum16(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
      if (lane == 15) {
        const int64_t r = r0 + j;
        theta[r] = ct.acc ? theta[r] + sq : sq;
      }
    }
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
  if constexpr (sizeof(ZT) == 4) {
    const size_t gz = (size_t)d * (kGZStride + 1) * sizeof(float);
    if (gz <= 152 * 1024) {
      auto kern = rownorm_csr_grp_kernel<T>;
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)gz);
      if (e != hipSuccess) return e;
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu));
      kern<<<grid, kCsrThreads, gz, s>>>(v, row_ptr, col_idx, n, d, nnz, Z, th, ct);
      return hipGetLastError();
    }
  }
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
