// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Used for the n-independent contractions of the estimator: the Gaussian
// transform A~ = G (S A) of Algorithm 3, the Gram A~^T A~ that drives the
// column-pivoted factorisation, and the rank-nb Schur complement updates of
// that factorisation.  All are small next to the passes over A, so this is a
// plain LDS-tiled kernel: 64 x 64 output tile per workgroup of 4 waves
// (each wave a 32 x 32 quadrant = 2 x 2 MFMA blocks), K in steps of 32
// through double-buffered LDS with the next step's global loads in flight
// during the current step's MFMAs, optional split-K with a fixed-order
// reduction (deterministic bits).
//
// MFMA operand layout (16x16x4 f64, wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator element v of lane l is
// C[(l / 16) + 4 * v][l % 16] (measured on gfx950; the f32 and bf16 forms
// use row 4 * (l / 16) + v instead).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int kThreads = 256;
constexpr int kPerThread = BM * BK / kThreads;  // elements of each operand a thread stages per K step

// One K step of the A and B tiles held in registers between the global
// loads and the LDS stores (the loads of step s + 1 are in flight while the
// matrix cores work on step s).
struct Stage {
  double a[kPerThread];
  double b[kPerThread];
};

__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(__hip_bfloat16 x) { return (double)__bfloat162float(x); }

// TI: element type of both operands in memory (FP64, or FP32 / BF16 widened
// exactly to FP64 on load).
template <typename TI>
__device__ __forceinline__ void load_stage(Stage& st, int tid, int64_t m0, int64_t n0, int64_t k0, int64_t ke,
                                           int64_t M, int64_t N, const TI* __restrict__ A, int64_t sai,
                                           int64_t sak, const TI* __restrict__ B, int64_t sbk, int64_t sbj) {
  const bool a_kfast = (sak == 1);
  const bool b_jfast = (sbj == 1);
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int e = tid + kThreads * q;
    // consecutive threads walk the operand's contiguous index
    const int kk = a_kfast ? e % BK : e / BM;
    const int ii = a_kfast ? e / BK : e % BM;
    const int64_t gi = m0 + ii, gk = k0 + kk;
    st.a[q] = (gi < M && gk < ke) ? to_f64(A[gi * sai + gk * sak]) : 0.0;
    const int kb = b_jfast ? e / BN : e % BK;
    const int jj = b_jfast ? e % BN : e / BK;
    const int64_t gj = n0 + jj, gk2 = k0 + kb;
    st.b[q] = (gj < N && gk2 < ke) ? to_f64(B[gk2 * sbk + gj * sbj]) : 0.0;
  }
}

// LDS layouts of one K step of an operand (64 rows x BK), chosen so that
// both the staging stores (consecutive threads walk the operand's contiguous
// index) and the MFMA operand reads (16 consecutive rows or columns per
// 16-lane group, one k per group) are free of bank conflicts:
//  * operand contiguous in k (KF): [i][k] with a row stride of BK + 2
//    doubles (68 banks = 4 mod 64: the four k groups of an MFMA read land on
//    disjoint bank pairs);
//  * operand contiguous in i: [k][i ^ 16 (k odd)] with a row stride of 64
//    doubles (the swizzle moves the odd-k groups to the other 32 banks).
constexpr int kLdsOp = BM * (BK + 2);  // doubles per operand buffer (the larger layout)

template <bool KF>
__device__ __forceinline__ int lds_idx(int k, int i) {
  if constexpr (KF) return i * (BK + 2) + k;
  else return k * BM + (i ^ ((k & 1) << 4));
}

template <bool AK, bool BJ>
__device__ __forceinline__ void store_stage(const Stage& st, int tid, double* __restrict__ As,
                                            double* __restrict__ Bs) {
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int e = tid + kThreads * q;
    const int kk = AK ? e % BK : e / BM;
    const int ii = AK ? e / BK : e % BM;
    As[lds_idx<AK>(kk, ii)] = st.a[q];
    const int kb = BJ ? e / BN : e % BK;
    const int jj = BJ ? e % BN : e / BK;
    Bs[lds_idx<!BJ>(kb, jj)] = st.b[q];
  }
}

// AK: A is contiguous in k (sak == 1); BJ: B is contiguous in j (sbj == 1).
// UPPER: C is symmetric (a Gram matrix): only the tiles on and above the
// diagonal run, on a one-dimensional grid of (upper tiles) x splits
// workgroups (workgroup w = split w / T, upper tile w % T in row order, T
// the number of upper tiles), so that consecutive workgroups, which go to
// consecutive XCDs, spread the triangle evenly over them (on a square grid
// the XCD of a tile is its row index mod 8, and the triangle loads the low
// XCDs up to twice as much as the high ones); with one split each upper tile
// is also stored transposed.
template <bool AK, bool BJ, typename TI = double, bool UPPER = false>
__global__ __launch_bounds__(kThreads) void dgemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                         const TI* __restrict__ A, int64_t sai,
                                                         int64_t sak, const TI* __restrict__ B,
                                                         int64_t sbk, int64_t sbj, double beta,
                                                         double* __restrict__ C, int64_t ldc, int splits,
                                                         int64_t kchunk, double* __restrict__ partial,
                                                         const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  __shared__ double As[2][kLdsOp];
  __shared__ double Bs[2][kLdsOp];

  int64_t bi = blockIdx.x, bj = blockIdx.y, bz = blockIdx.z;
  if constexpr (UPPER) {
    const int64_t tb = (M + BM - 1) / BM;  // M == N
    const int64_t T = tb * (tb + 1) / 2;
    bz = (int64_t)blockIdx.x / T;
    int64_t t = (int64_t)blockIdx.x % T, I = 0;
    while (t >= tb - I) {  // row I of the triangle holds tb - I tiles
      t -= tb - I;
      ++I;
    }
    bi = I;
    bj = I + t;
  }
  const int64_t m0 = bi * BM;
  const int64_t n0 = bj * BN;
  const int64_t kb = bz * kchunk;
  const int64_t ke = std::min<int64_t>(K, kb + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  Stage st;
  int buf = 0;
  if (kb < ke) {
    load_stage(st, tid, m0, n0, kb, ke, M, N, A, sai, sak, B, sbk, sbj);
    store_stage<AK, BJ>(st, tid, As[0], Bs[0]);
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;  // uniform
    if (more) load_stage(st, tid, m0, n0, k0 + BK, ke, M, N, A, sai, sak, B, sbk, sbj);
    // the operands of group g + 1 are read before the MFMAs of group g are
    // issued, so the LDS latency hides behind them
    double a[2][2], b[2][2];
    auto read_group = [&](int k4, int slot) {
#pragma unroll
      for (int i = 0; i < 2; ++i) a[slot][i] = As[buf][lds_idx<AK>(k4 + (lane >> 4), wm + 16 * i + (lane & 15))];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[slot][j] = Bs[buf][lds_idx<!BJ>(k4 + (lane >> 4), wn + 16 * j + (lane & 15))];
    };
    read_group(0, 0);
#pragma unroll
    for (int k4 = 0; k4 < BK; k4 += 4) {
      const int cur = (k4 / 4) & 1;
      if (k4 + 4 < BK) read_group(k4 + 4, cur ^ 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // the other buffer was last read before the previous barrier
    if (more) store_stage<AK, BJ>(st, tid, As[buf ^ 1], Bs[buf ^ 1]);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = m0 + wm + 16 * i + (lane >> 4) + 4 * v;
        const int64_t gj = n0 + wn + 16 * j + (lane & 15);
        if (gi < M && gj < N) {
          if (splits == 1) {
            const double prev = (beta != 0.0) ? beta * C[gi * ldc + gj] : 0.0;
            C[gi * ldc + gj] = alpha * acc[i][j][v] + prev;
            if (UPPER) C[gj * ldc + gi] = alpha * acc[i][j][v] + prev;
          } else {
            partial[(bz * M + gi) * N + gj] = acc[i][j][v];
          }
        }
      }
}

__global__ void splitk_reduce_kernel(int64_t M, int64_t N, int splits, const double* __restrict__ partial,
                                     double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                     const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx / N, j = idx % N;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[(int64_t)z * M * N + idx];
  const double prev = (beta != 0.0) ? beta * C[i * ldc + j] : 0.0;
  C[i * ldc + j] = alpha * s + prev;
}

// Gram form of the split-K sum: C[i][j] from the partial of the upper
// tile holding (i, j) or (j, i).
// C = the sum of the split partials of the upper tiles, mirrored below the
// diagonal: workgroup t takes upper tile (I, J) (row order over the
// triangle), sums its partials in split order with reads along j, writes
// the tile and, through LDS, its transpose with writes along j as well.
// Diagonal tiles keep each element as summed.
__global__ __launch_bounds__(1024) void gram_reduce_kernel(int64_t N, int splits, const double* __restrict__ partial,
                                                           double* __restrict__ C) {
  __shared__ double tile[BM][BM + 1];
  const int64_t tb = (N + BM - 1) / BM;
  int64_t t = blockIdx.x, I = 0;
  while (t >= tb - I) {
    t -= tb - I;
    ++I;
  }
  const int64_t J = I + t, i0 = I * BM, j0 = J * BM;
  const int jj = threadIdx.x % BM, r0 = threadIdx.x / BM;  // 16 rows per pass
  for (int ii = r0; ii < BM; ii += 1024 / BM) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    double acc = 0.0;
    if (gi < N && gj < N)
      for (int z = 0; z < splits; ++z) acc += partial[((int64_t)z * N + gi) * N + gj];
    tile[ii][jj] = acc;
  }
  __syncthreads();
  for (int ii = r0; ii < BM; ii += 1024 / BM) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < N && gj < N) C[gi * N + gj] = tile[ii][jj];
    const int64_t ti = j0 + ii, tj = i0 + jj;  // row j0 + ii of the tile below the diagonal
    if (I < J && ti < N && tj < N) C[ti * N + tj] = tile[jj][ii];
  }
}

}  // namespace

int dgemm_choose_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int splits = 1;
  // Aim for >= 512 workgroups (2 per CU) while each split keeps >= 64 of K
  // (two K steps, so the prefetch of the second has the first to hide
  // behind): a short-K product like the 256 x 256 Gram of a 512-row sketch
  // then spreads over 128 workgroups instead of 32.
  while (tiles * splits < 512 && K / (splits * 2) >= 64 && splits < 64) splits *= 2;
  return splits;
}

size_t dgemm_partial_elems(int64_t M, int64_t N, int splits) {
  return splits > 1 ? (size_t)splits * (size_t)M * (size_t)N : 0;
}

hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sai,
                        int64_t sak, const double* B, int64_t sbk, int64_t sbj, double beta,
                        double* C, int64_t ldc, int splits, double* partial, const int32_t* skip,
                        hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk == 0) kchunk = BK;
  dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)splits);
  const bool ak = (sak == 1), bj = (sbj == 1);
  auto kern = ak ? (bj ? dgemm_kernel<true, true> : dgemm_kernel<true, false>)
                 : (bj ? dgemm_kernel<false, true> : dgemm_kernel<false, false>);
  kern<<<grid, kThreads, 0, s>>>(M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, ldc, splits, kchunk, partial,
                                 skip);
  if (splits > 1) {
    const int64_t total = M * N;
    splitk_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(M, N, splits, partial, alpha,
                                                                          beta, C, ldc, skip);
  }
  return hipGetLastError();
}

// The Gram's K is the row count n: long, while only the tiles on and above
// the diagonal run.  Aim for >= 2048 workgroups (eight per CU: each K step is
// a global-load round trip that the other workgroups' MFMAs cover) with
// >= 512 rows per split and the partials within 64 MiB (d = 64: 1024 splits;
// d = 256: 128; d = 1024: 8).
int gram_dense_splits(int64_t n, int64_t d) {
  const int64_t tb = (d + BM - 1) / BM;
  const int64_t upper = tb * (tb + 1) / 2;
  const int64_t cap = std::max<int64_t>(1, (int64_t(64) << 20) / (8 * d * d));
  int splits = 1;
  while (upper * splits < 2048 && n / (splits * 2) >= 512 && splits * 2 <= cap && splits < 1024) splits *= 2;
  return splits;
}

// A^T A: op(A)[i][k] = A[k][i] (strides 1, ld) and op(B)[k][j] = A[k][j]
// (strides ld, 1), so both operand tiles are read along A's rows; only the
// tiles on and above the diagonal are computed.
hipError_t launch_gram_dense(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int splits,
                             double* partial, double* B, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int64_t kchunk = (n + splits - 1) / splits;
  kchunk = std::max<int64_t>(BK, ((kchunk + BK - 1) / BK) * BK);
  const int64_t tb = (d + BM - 1) / BM;
  const dim3 grid((unsigned)(tb * (tb + 1) / 2 * splits));  // upper tiles x splits (see dgemm_kernel)
  switch (dtype) {
    case 0:
      dgemm_kernel<false, true, double, true><<<grid, kThreads, 0, s>>>(d, d, n, 1.0, static_cast<const double*>(A),
                                                                        1, ld, static_cast<const double*>(A), ld, 1,
                                                                        0.0, B, d, splits, kchunk, partial, nullptr);
      break;
    case 1:
      dgemm_kernel<false, true, float, true><<<grid, kThreads, 0, s>>>(d, d, n, 1.0, static_cast<const float*>(A), 1,
                                                                       ld, static_cast<const float*>(A), ld, 1, 0.0,
                                                                       B, d, splits, kchunk, partial, nullptr);
      break;
    case 2: {
      const auto* a = static_cast<const __hip_bfloat16*>(A);
      dgemm_kernel<false, true, __hip_bfloat16, true><<<grid, kThreads, 0, s>>>(d, d, n, 1.0, a, 1, ld, a, ld, 1, 0.0,
                                                                                B, d, splits, kchunk, partial,
                                                                                nullptr);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  if (splits > 1) gram_reduce_kernel<<<(unsigned)(tb * (tb + 1) / 2), 1024, 0, s>>>(d, splits, partial, B);
  return hipGetLastError();
}

// Splits of the sketch's Gram A~^T A~ (m rows) on the upper tiles: as many
// as keep every workgroup in one round at two per CU with at least 64 of the
// rows each, and at least two, so that the sums always go through the
// partials and the lower half is the mirror of the upper one.
int gram_sketch_splits(int64_t m, int64_t d) {
  const int64_t tb = (d + BM - 1) / BM;
  const int64_t upper = tb * (tb + 1) / 2;
  int splits = 2;
  while (upper * (splits + 1) <= 512 && m / (splits + 1) >= 64 && splits < 64) ++splits;
  return splits;
}

}  // namespace lev
