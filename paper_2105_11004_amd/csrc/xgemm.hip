// The Gaussian transform A~ = G (S A) of Algorithm 3 in FP32-level
// arithmetic on the BF16 matrix cores, for BF16-stored A.
//
// Both operands are split exactly into three BF16 parts (hi + mid + lo,
// 24 significant bits, like FP32): G while pass 1 draws it (the side draw
// writes the parts instead of FP64 values), S A by split_t3_kernel below,
// which also transposes it so that both operands are contiguous in the
// contraction index.  The six part products above 2^-24 relative (hh, hm,
// mh, hl, mm, lh) run on 16x16x32 BF16 MFMAs; each 32-wide K step of them is
// summed in FP32 and added into FP64 accumulators, so FP32 rounding only
// ever sums 192 products of one K step.  A~ then carries relative error
// ~2^-24 against the FP64 product (the FP64 transform takes the GEMM at the
// FP64 matrix rate, ~25x slower than this on gfx950).
//
// Tiling: 128 x 128 output tile per workgroup of 8 waves (each wave 64 rows
// x 32 columns = 4 x 2 MFMA blocks), K in steps of 32 through
// double-buffered LDS (3 parts x 128 rows x 32 k per operand, the k pieces
// of each row swizzled against bank conflicts), the next two steps' global
// loads in registers while the current step's MFMAs run, optional split-K
// with partials reduced in a
// fixed order.  Workgroups that share an A tile are placed on the same XCD
// (blockIdx % 8) so that its re-reads hit that die's L2.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kRowHalfs = 32;  // LDS row stride in BF16 elements (64 bytes, unpadded)
// Position (in BF16 elements) of 16-byte k piece pc of tile row r in its LDS
// row: the pieces are XOR-swizzled by (r / 2) mod 4, so that both the
// staging stores (4 rows x 64 bytes per 16 lanes) and the MFMA operand reads
// (16 rows at one k piece) hit distinct banks (measured on gfx950: no bank
// conflicts, against 5 conflict cycles per LDS instruction with 80-byte
// padded rows and 2-3 with other swizzles or paddings).
__device__ __forceinline__ int xg_piece(int r, int pc) { return 8 * (pc ^ ((r >> 1) & 3)); }
constexpr int kPieces = 2 * 3 * TM * (TK / 8);       // 16-byte pieces per K step (A and B)
constexpr int kPer = kPieces / kThreads;             // 6 per thread
constexpr int kOpHalfs = 3 * TM * kRowHalfs;         // BF16 elements per operand buffer

__device__ __forceinline__ v8bf as_bf(const uint4& u) { return __builtin_bit_cast(v8bf, u); }

// Workgroup barrier that orders LDS traffic only: __syncthreads() would also
// wait for the staged loads of the next two steps.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}

// x = h + m + l exactly in FP32 for two values, parts packed in pairs.
__device__ __forceinline__ void split3_pair(float x0, float x1, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = pk_bf16(x0, x1);
  const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xFFFF0000u);
  m = pk_bf16(r0, r1);
  const float s0 = r0 - __uint_as_float(m << 16), s1 = r1 - __uint_as_float(m & 0xFFFF0000u);
  l = pk_bf16(s0, s1);
}

// out part p (N x K, BF16, row-major: contiguous in k) = split(SA^T), SA
// K x N row-major (FP64, or FP32 as pass 1 stores it for this transform).
// A 64 x 64 tile goes through LDS (as FP32: the split starts from the FP32
// value) so that both the reads (along j) and the writes (pairs of k along
// k) are coalesced.
constexpr int kT = 64;
template <typename TS>
__global__ __launch_bounds__(256) void split_t3_kernel(int64_t K, int64_t N, const TS* __restrict__ SA,
                                                       uint32_t* __restrict__ out) {
  __shared__ float tile[kT][kT + 1];
  const int64_t Kp = (K + 1) / 2;
  const int64_t k0 = (int64_t)blockIdx.x * kT, j0 = (int64_t)blockIdx.y * kT;
  const int t = threadIdx.x;
  // read: thread t covers column j0 + t % 64 of rows k0 + t / 64 + 4 r
#pragma unroll 4
  for (int r = 0; r < kT / 4; ++r) {
    const int kk = t / kT + 4 * r, jj = t % kT;
    const int64_t k = k0 + kk, j = j0 + jj;
    tile[kk][jj] = (k < K && j < N) ? (float)SA[k * N + j] : 0.0f;
  }
  __syncthreads();
  // write: thread t covers pair kp0 + t % 32 of columns j0 + t / 32 + 8 r
#pragma unroll 4
  for (int r = 0; r < kT / 8; ++r) {
    const int pp = t % (kT / 2), jj = t / (kT / 2) + 8 * r;
    const int64_t kp = k0 / 2 + pp, j = j0 + jj;
    if (kp < Kp && j < N) {
      uint32_t h, m, l;
      split3_pair(tile[2 * pp][jj], tile[2 * pp + 1][jj], h, m, l);
      const int64_t o = j * Kp + kp;
      out[o] = h;
      out[Kp * N + o] = m;
      out[2 * Kp * N + o] = l;
    }
  }
}

// C or partial[z] (M x N FP64) = sum over the products of A part p (M x K)
// times B part q (N x K), K range of split z.  Ap, Bp: 3 parts one after
// the other, each `pstride` BF16 elements, rows of ldk elements.
__global__ __launch_bounds__(kThreads, 1) void xgemm_kernel(int64_t M, int64_t N, int64_t K, int64_t ldk,
                                                            const __hip_bfloat16* __restrict__ Ap, int64_t apstride,
                                                            const __hip_bfloat16* __restrict__ Bp, int64_t bpstride,
                                                            double* __restrict__ C, int64_t ldc, int splits,
                                                            int64_t kchunk, double* __restrict__ partial) {
  __shared__ __align__(16) __hip_bfloat16 As[2][kOpHalfs];
  __shared__ __align__(16) __hip_bfloat16 Bs[2][kOpHalfs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // XCD-aware placement: the 8 column tiles of one (row tile, split) pair
  // run on one XCD (blockIdx % 8), so its A tile is re-read from that L2
  const int64_t mt = (M + TM - 1) / TM, ntl = (N + TN - 1) / TN;
  const int64_t nwg = (int64_t)gridDim.x;
  int64_t id = blockIdx.x;
  int64_t pair, nt_i;
  if (ntl == 8 && nwg % 64 == 0) {  // (row tile, split) pairs a multiple of 8
    const int64_t xcd = id % 8, j = id / 8;
    pair = (nwg / 64) * xcd + j / 8;  // (row tile, split) pairs of this XCD
    nt_i = j % 8;
  } else {
    pair = id / ntl;
    nt_i = id % ntl;
  }
  const int64_t z = pair % splits, mt_i = pair / splits;
  if (mt_i >= mt) return;
  const int64_t m0 = mt_i * TM, n0 = nt_i * TN;
  const int64_t kb = z * kchunk;
  const int64_t ke = std::min<int64_t>(K, kb + kchunk);
  const int wm = (wave >> 2) * 64, wn = (wave & 3) * 32;

  // staging: piece e = tid + kThreads * q; operand e / (kPieces / 2), part,
  // row and 16-byte k piece within the step.  Two steps' pieces are in
  // flight in registers (stgA, stgB alternate) while a third is multiplied
  // from LDS: one step's products (≈0.6 µs of MFMA work per SIMD) do not
  // cover an L2 round trip, two do.  Loads past the range read a valid
  // address and are zeroed when stored to LDS, so no branch or select
  // touches a loaded value before it is needed (either would make the
  // compiler wait for the load there).
  // Per staged piece q (operand q / 3 by construction: tid < kThreads and
  // kPieces / 2 = 3 kThreads): its operand row pointer at its k piece (the
  // row clamped to a valid one) and its place in an LDS buffer.  Whole
  // tiles and whole K steps (uniform tests) load and store with no
  // predicate; the masked forms below take the rest.
  const bool rows_full = m0 + TM <= M && n0 + TN <= N;
  const __hip_bfloat16* qptr[kPer];
  int qlds[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + kThreads * q;
    const int op = e / (kPieces / 2), ee = e % (kPieces / 2);
    const int part = ee / (TM * 4), row = (ee % (TM * 4)) / 4, pc = ee % 4;
    const __hip_bfloat16* base = op == 0 ? Ap + part * apstride : Bp + part * bpstride;
    const int64_t gr = (op == 0 ? m0 : n0) + row;
    qptr[q] = base + (gr < (op == 0 ? M : N) ? gr : 0) * ldk + 8 * pc;
    qlds[q] = (part * TM + row) * kRowHalfs + xg_piece(row, pc);
  }
#define LEV_XG_FAST(K0) (rows_full && (K0) + TK <= ke)
#define LEV_XG_LOAD_FAST(STG, K0)                                                                     \
  _Pragma("unroll") for (int q = 0; q < kPer; ++q) STG[q] = *reinterpret_cast<const uint4*>(qptr[q] + (K0));
#define LEV_XG_STORE_FAST(STG, BUF)                                                                   \
  _Pragma("unroll") for (int q = 0; q < kPer; ++q)                                                    \
    *reinterpret_cast<uint4*>((q < kPer / 2 ? As[BUF] : Bs[BUF]) + qlds[q]) = STG[q];
#define LEV_XG_LOAD(STG, K0)                                                                          \
  _Pragma("unroll") for (int q = 0; q < kPer; ++q) {                                                  \
    const int e = tid + kThreads * q;                                                                 \
    const int op = e / (kPieces / 2), ee = e % (kPieces / 2);                                         \
    const int part = ee / (TM * 4), row = (ee % (TM * 4)) / 4, pc = ee % 4;                           \
    const int64_t gk = (K0) + 8 * pc;                                                                 \
    const __hip_bfloat16* base = op == 0 ? Ap + part * apstride : Bp + part * bpstride;               \
    const int64_t gr = (op == 0 ? m0 : n0) + row;                                                     \
    const int64_t lim = op == 0 ? M : N;                                                              \
    const bool ok = gr < lim && gk < ke; /* else a valid address, zeroed at the store */              \
    STG[q] = *reinterpret_cast<const uint4*>(base + (ok ? gr : 0) * ldk + (ok ? gk : 0));             \
  }
/* pieces outside the operand or the K range go to LDS as zeros (masked at
   the store, where the data is needed anyway, so no earlier wait) */
#define LEV_XG_STORE(STG, BUF, K0)                                                                    \
  _Pragma("unroll") for (int q = 0; q < kPer; ++q) {                                                  \
    const int e = tid + kThreads * q;                                                                 \
    const int op = e / (kPieces / 2), ee = e % (kPieces / 2);                                         \
    const int part = ee / (TM * 4), row = (ee % (TM * 4)) / 4, pc = ee % 4;                           \
    const int64_t gk = (K0) + 8 * pc;                                                                 \
    const int64_t gr = (op == 0 ? m0 : n0) + row;                                                     \
    const bool ok = gr < (op == 0 ? M : N) && gk < ke;                                                \
    __hip_bfloat16* dst = (op == 0 ? As[BUF] : Bs[BUF]) + (part * TM + row) * kRowHalfs + xg_piece(row, pc); \
    *reinterpret_cast<uint4*>(dst) = ok ? STG[q] : make_uint4(0u, 0u, 0u, 0u);                        \
  }

  v4f acc[4][2];
  double acc64[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }

// (the empty asm pins each FP64 sum where it is written: otherwise the
// compiler sinks all the adds below the step's last MFMA)
#define LEV_XG_FLUSH(I)                                                                               \
  _Pragma("unroll") for (int j = 0; j < 2; ++j)                                                       \
  _Pragma("unroll") for (int v = 0; v < 4; ++v) {                                                     \
    acc64[I][j][v] += (double)acc[I][j][v];                                                           \
    asm volatile("" : "+v"(acc64[I][j][v]));                                                          \
  }

  // B fragments of the wave's two column blocks (all parts), then per row
  // block the A fragments and the six products, smallest first, the first
  // from a zero accumulator.  A row block's FP32 sums go into FP64 once the
  // next row block's products are issued (its own have finished by then),
  // so the conversions and FP64 adds sit between MFMAs and only the last
  // row block's wait at the end of the step; the FP64 sums take the steps
  // in order either way.
#define LEV_XG_AFRAG(BUF, I, DST)                                                                     \
  _Pragma("unroll") for (int p = 0; p < 3; ++p)                                                       \
    DST[p] = *reinterpret_cast<const uint4*>(As[BUF] + (p * TM + wm + 16 * (I) + (lane & 15)) * kRowHalfs + \
                                             xg_piece(wm + 16 * (I) + (lane & 15), lane >> 4));
#define LEV_XG_COMPUTE(BUF)                                                                           \
  {                                                                                                   \
    uint4 bq[2][3];                                                                                   \
    _Pragma("unroll") for (int j = 0; j < 2; ++j)                                                     \
    _Pragma("unroll") for (int p = 0; p < 3; ++p)                                                     \
      bq[j][p] = *reinterpret_cast<const uint4*>(Bs[BUF] + (p * TM + wn + 16 * j + (lane & 15)) * kRowHalfs + \
                                                 xg_piece(wn + 16 * j + (lane & 15), lane >> 4));     \
    uint4 ap[3], apn[3];                                                                              \
    LEV_XG_AFRAG(BUF, 0, ap)                                                                          \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                                   \
      if (i < 3) { LEV_XG_AFRAG(BUF, i + 1, apn) }                                                    \
      _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                                 \
        v4f c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[2]), as_bf(bq[j][0]),                \
                                                        (v4f{0.f, 0.f, 0.f, 0.f}), 0, 0, 0);         \
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[1]), as_bf(bq[j][1]), c, 0, 0, 0);      \
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[0]), as_bf(bq[j][2]), c, 0, 0, 0);      \
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[1]), as_bf(bq[j][0]), c, 0, 0, 0);      \
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[0]), as_bf(bq[j][1]), c, 0, 0, 0);      \
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ap[0]), as_bf(bq[j][0]), c, 0, 0, 0);      \
        acc[i][j] = c;                                                                                \
      }                                                                                               \
      if (i > 0) { LEV_XG_FLUSH(i - 1) }                                                              \
      /* keeps the flush of row block i - 1 among row block i's MFMAs */                              \
      __builtin_amdgcn_sched_barrier(0);                                                              \
      _Pragma("unroll") for (int p = 0; p < 3; ++p) ap[p] = apn[p];                                   \
    }                                                                                                 \
    LEV_XG_FLUSH(3)                                                                                   \
  }

  // (the products are l h, m m, h l, m h, h m, h h: smallest first)
  const int64_t nsteps = ke > kb ? (ke - kb + TK - 1) / TK : 0;
  uint4 stgA[kPer], stgB[kPer];
#define LEV_XG_LOAD_ANY(STG, K0)                                                                      \
  if (LEV_XG_FAST(K0)) {                                                                              \
    LEV_XG_LOAD_FAST(STG, K0)                                                                         \
  } else {                                                                                            \
    LEV_XG_LOAD(STG, K0)                                                                              \
  }
#define LEV_XG_STORE_ANY(STG, BUF, K0)                                                                \
  if (LEV_XG_FAST(K0)) {                                                                              \
    LEV_XG_STORE_FAST(STG, BUF)                                                                       \
  } else {                                                                                            \
    LEV_XG_STORE(STG, BUF, K0)                                                                        \
  }
  LEV_XG_LOAD_ANY(stgA, kb)
  LEV_XG_STORE_ANY(stgA, 0, kb)
  LEV_XG_LOAD_ANY(stgB, kb + TK)
  __syncthreads();
  for (int64_t s = 0; s < nsteps; s += 2) {
    // step s from buffer 0; step s + 1 is in stgB; step s + 2 into stgA
    LEV_XG_LOAD_ANY(stgA, kb + (s + 2) * TK)
    LEV_XG_COMPUTE(0)
    LEV_XG_STORE_ANY(stgB, 1, kb + (s + 1) * TK)  // buffer 1 was last read before the previous barrier
    lds_barrier();
    if (s + 1 >= nsteps) break;  // uniform
    // step s + 1 from buffer 1; step s + 2 is in stgA; step s + 3 into stgB
    LEV_XG_LOAD_ANY(stgB, kb + (s + 3) * TK)
    LEV_XG_COMPUTE(1)
    LEV_XG_STORE_ANY(stgA, 0, kb + (s + 2) * TK)  // buffer 0 was last read before the barrier above
    lds_barrier();
  }
#undef LEV_XG_LOAD_ANY
#undef LEV_XG_STORE_ANY
#undef LEV_XG_LOAD_FAST
#undef LEV_XG_STORE_FAST
#undef LEV_XG_FAST
#undef LEV_XG_LOAD
#undef LEV_XG_STORE
#undef LEV_XG_COMPUTE
#undef LEV_XG_FLUSH
#undef LEV_XG_AFRAG

  // accumulator element v of lane l: row 4 (l / 16) + v, column l % 16 of
  // its 16 x 16 block
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int64_t gj = n0 + wn + 16 * j + (lane & 15);
        if (gi < M && gj < N) {
          if (splits == 1) C[gi * ldc + gj] = acc64[i][j][v];
          else partial[(z * M + gi) * N + gj] = acc64[i][j][v];
        }
      }
}

__global__ void xgemm_reduce_kernel(int64_t M, int64_t N, int splits, const double* __restrict__ partial,
                                    double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[(int64_t)z * M * N + idx];
  C[(idx / N) * ldc + idx % N] = s;
}

}  // namespace

int xgemm_choose_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  int splits = 1;
  // about one workgroup per CU (one fits: its LDS is 120 KB), each split
  // keeping at least 16 K steps
  while (tiles * splits < 256 && K / (splits * 2) >= 16 * TK && splits < 64) splits *= 2;
  return splits;
}

size_t xgemm_partial_elems(int64_t M, int64_t N, int splits) {
  return splits > 1 ? (size_t)splits * (size_t)M * (size_t)N : 0;
}

size_t split3_elems(int64_t rows, int64_t K) { return (size_t)rows * (size_t)((K + 1) / 2) * 2; }

hipError_t launch_split_t3(int64_t K, int64_t N, const void* SA, bool sa_f32, void* out, hipStream_t s) {
  if (K <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((K + kT - 1) / kT), (unsigned)((N + kT - 1) / kT));
  if (sa_f32)
    split_t3_kernel<float><<<grid, 256, 0, s>>>(K, N, static_cast<const float*>(SA), static_cast<uint32_t*>(out));
  else
    split_t3_kernel<double><<<grid, 256, 0, s>>>(K, N, static_cast<const double*>(SA), static_cast<uint32_t*>(out));
  return hipGetLastError();
}

hipError_t launch_xgemm(int64_t M, int64_t N, int64_t K, const void* Ap, const void* Bp, double* C, int64_t ldc,
                        int splits, double* partial, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K % 8 != 0) return hipErrorInvalidValue;  // 16-byte pieces of k
  if (splits < 1) splits = 1;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + TK - 1) / TK * TK;
  const int64_t ldk = K;  // rows of the parts are exactly K elements (K even)
  const int64_t apstride = M * ldk, bpstride = N * ldk;
  const int64_t pairs = ((M + TM - 1) / TM) * splits;
  const int64_t ntl = (N + TN - 1) / TN;
  xgemm_kernel<<<(unsigned)(pairs * ntl), kThreads, 0, s>>>(
      M, N, K, ldk, static_cast<const __hip_bfloat16*>(Ap), apstride, static_cast<const __hip_bfloat16*>(Bp),
      bpstride, C, ldc, splits, kchunk, partial);
  if (splits > 1) {
    const int64_t total = M * N;
    xgemm_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(M, N, splits, partial, C, ldc);
  }
  return hipGetLastError();
}

}  // namespace lev
