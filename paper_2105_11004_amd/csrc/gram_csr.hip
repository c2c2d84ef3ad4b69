// B = A^T A for CSR A in sum_i nnz_i^2 work: the Gram route of Algorithm 5
// (and of Algorithm 7's exact scores), which costs the square of each row's
// nonzero count instead of d^2 per row.
//
// Row i adds the outer product a_i a_i^T, i.e. a_ip a_iq at (c_p, c_q) for
// every pair of its nonzeros.  B is cut into 128 x 128 tiles (I, J), I <= J
// (B is symmetric); a workgroup owns one tile in LDS (FP64, rows padded to
// kGS doubles so that the rows of one atomic instruction spread over the
// banks) and one chunk of rows.  A wave takes one row at a time: column ids
// are sorted within a row, so the entries in block I and in block J are two
// contiguous runs, found by counting ids below the block bounds (a wave
// walks 64 rows at a time with their extents in one load, and a row of at
// most 64 entries is read once, the next row's read in flight, and its
// pairs of run entries go one per lane, 64 per atomic instruction); a longer
// row's lanes hold its runs (up to 128 entries each, two per lane) and, for
// each entry p
// of run I in turn (its id and value read from the holding lane), add
// a_ip a_iq for the entries q of run J, one per lane, by LDS atomic adds.
// On a diagonal tile only q >= p is added (the upper triangle, mirrored when
// the tiles are summed).  The tiles of all chunks are summed in chunk order
// into B and mirrored below the diagonal.  FP32 and BF16 values give exact
// FP64 products; the order of the atomic adds inside a workgroup is not
// fixed, so B's last bits can vary between runs.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kGT = 128;             // tile edge
constexpr int kGS = kGT + 1;         // LDS row stride of the tile, in doubles
constexpr int kGThreads = 1024;      // 16 waves
constexpr int kGWaves = kGThreads / 64;
constexpr int kTargetGroups = 512;   // workgroups per launch (one per CU resident: 129 KB of LDS)
constexpr size_t kTileBytes = sizeof(double) * kGT * kGS;

__device__ __forceinline__ double val_f64(double x) { return x; }
__device__ __forceinline__ double val_f64(float x) { return (double)x; }
__device__ __forceinline__ double val_f64(__hip_bfloat16 x) { return (double)__bfloat162float(x); }

int64_t blocks_per_side(int64_t d) { return (d + kGT - 1) / kGT; }
int64_t tile_pairs(int64_t d) {
  const int64_t nb = blocks_per_side(d);
  return nb * (nb + 1) / 2;
}
int64_t row_chunks(int64_t n, int64_t d) {
  const int64_t want = (kTargetGroups + tile_pairs(d) - 1) / tile_pairs(d);
  return std::max<int64_t>(1, std::min<int64_t>(want, (n + 255) / 256));
}

// Tile pair q (0 <= q < nb (nb + 1) / 2) -> (I, J), I <= J, row-major over
// the upper triangle.
__device__ __forceinline__ void pair_of(int q, int nb, int& I, int& J) {
  int i = 0, left = q;
  while (left >= nb - i) {
    left -= nb - i;
    ++i;
  }
  I = i;
  J = i + left;
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <typename T>
__global__ __launch_bounds__(kGThreads) void gram_csr_kernel(const T* __restrict__ vals,
                                                             const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ col_idx, int64_t n,
                                                             int64_t d, int64_t nnz, int64_t rows_per_chunk,
                                                             double* __restrict__ partial) {
  extern __shared__ double tile[];  // kGT rows of kGS
  const int nb = (int)((d + kGT - 1) / kGT);
  int I, J;
  pair_of((int)blockIdx.x, nb, I, J);
  const bool diag = I == J;
  const int32_t I0 = I * kGT, J0 = J * kGT;
  const int32_t Iend = (int32_t)std::min<int64_t>(d, I0 + kGT), Jend = (int32_t)std::min<int64_t>(d, J0 + kGT);
  for (int e = threadIdx.x; e < kGT * kGS; e += kGThreads) tile[e] = 0.0;
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
  // The pairs of one row with its entries in registers: entry t (t < lI of
  // run I, t < lJ of run J) held by lane t % 64, slot t / 64.
  auto add_pairs = [&](const int32_t (&cI)[2], const double (&vI)[2], const int32_t (&cJ)[2],
                       const double (&vJ)[2], int lI) {
    for (int p = 0; p < lI; ++p) {
      const int h = p >> 6, l = p & 63;
      const int32_t cp = __builtin_amdgcn_readlane(h ? cI[1] : cI[0], l);
      const double vp = readlane_f64(h ? vI[1] : vI[0], l);
      if ((uint32_t)cp >= (uint32_t)kGT) continue;
      double* row = tile + cp * kGS;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        // diagonal tile: the upper triangle (q >= p, i.e. c_q >= c_p) only
        if (cJ[q] >= 0 && (!diag || cJ[q] >= cp)) atomicAdd(row + cJ[q], vp * vJ[q]);
      }
    }
  };
  // A wave takes 64 consecutive rows at a time: their extents in one load
  // (lane j: row i0 + j), then row by row.  A row of at most 64 entries is
  // loaded once (ids and values, one per lane, the next row's load in
  // flight while this row's pairs are added) and its pairs of run entries
  // are dealt out one per lane; longer rows count and load their runs from
  // memory in 64-entry pieces.
  for (int64_t i0 = r0 + 64 * (int64_t)wave; i0 < r1; i0 += 64 * (int64_t)kGWaves) {
    const int nr = (int)std::min<int64_t>(64, r1 - i0);
    // row extents clamped to [0, nnz] and made non-decreasing (a malformed
    // row_ptr gives a wrong B, no stray access)
    int64_t rs = lane < nr ? std::min<int64_t>(std::max<int64_t>(row_ptr[i0 + lane], 0), nnz) : nnz;
    int64_t re = lane < nr ? std::min<int64_t>(std::max<int64_t>(row_ptr[i0 + lane + 1], 0), nnz) : nnz;
    re = std::max(re, rs);
    auto load_short = [&](int j, int32_t& c, double& v) {
      // entry `lane` of row j when the row has at most 64 entries
      const int64_t s = ((int64_t)__builtin_amdgcn_readlane((int)(rs >> 32), j) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)rs, j);
      const int64_t e = ((int64_t)__builtin_amdgcn_readlane((int)(re >> 32), j) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)re, j);
      const bool ok = e - s <= 64 && s + lane < e;
      c = ok ? col_idx[s + lane] : INT32_MAX;
      v = ok ? val_f64(vals[s + lane]) : 0.0;
    };
    int32_t nc;
    double nv;
    load_short(0, nc, nv);
    for (int j = 0; j < nr; ++j) {
      const int32_t c = nc;
      const double v = nv;
      if (j + 1 < nr) load_short(j + 1, nc, nv);
      const int64_t s = ((int64_t)__builtin_amdgcn_readlane((int)(rs >> 32), j) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)rs, j);
      const int64_t e = ((int64_t)__builtin_amdgcn_readlane((int)(re >> 32), j) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)re, j);
      const int64_t len = e - s;
      if (len == 0) continue;
      if (len <= 64) {
        // positions of the runs [I0, Iend) and [J0, Jend) among the sorted ids
        const int loI = __popcll(__ballot(c < I0)), hiI = __popcll(__ballot(c < Iend));
        const int loJ = __popcll(__ballot(c < J0)), hiJ = __popcll(__ballot(c < Jend));
        const int lI = hiI - loI, lJ = hiJ - loJ;
        if (lI <= 0 || lJ <= 0) continue;
        // one lane per pair (p, q) of the two runs, 64 pairs per step: the
        // entries come from their lanes by shuffles that every lane takes
        // part in
        const int np = lI * lJ;
        for (int k0 = 0; k0 < np; k0 += 64) {
          const int k = k0 + lane;
          const int pp = k / lJ, qq = k - pp * lJ;
          const bool ok = k < np;
          const int srcp = ok ? loI + pp : 0, srcq = ok ? loJ + qq : 0;
          const int32_t cp = __shfl(c, srcp, 64) - I0, cq = __shfl(c, srcq, 64) - J0;
          const double vp = __shfl(v, srcp, 64), vq = __shfl(v, srcq, 64);
          // ids outside the blocks (an unsorted row) are dropped; on a
          // diagonal tile only the upper triangle (c_q >= c_p) is added
          if (ok && (uint32_t)cp < (uint32_t)kGT && (uint32_t)cq < (uint32_t)kGT && (!diag || cq >= cp))
            atomicAdd(tile + cp * kGS + cq, vp * vq);
        }
        continue;
      }
      int32_t cI[2], cJ[2];
      double vI[2], vJ[2];
      int loI = 0, hiI = 0, loJ = 0, hiJ = 0;
      for (int64_t c0 = s; c0 < e; c0 += 64) {
        const int64_t p = c0 + lane;
        const int32_t cc = p < e ? col_idx[p] : INT32_MAX;
        loI += __popcll(__ballot(cc < I0));
        hiI += __popcll(__ballot(cc < Iend));
        loJ += __popcll(__ballot(cc < J0));
        hiJ += __popcll(__ballot(cc < Jend));
      }
      const int lI = std::min(hiI - loI, kGT), lJ = std::min(hiJ - loJ, kGT);
      if (lI <= 0 || lJ <= 0) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        const int64_t pi = s + loI + t, pj = s + loJ + t;
        cI[h] = t < lI ? col_idx[pi] - I0 : 0;
        vI[h] = t < lI ? val_f64(vals[pi]) : 0.0;
        cJ[h] = t < lJ ? col_idx[pj] - J0 : -1;
        vJ[h] = t < lJ ? val_f64(vals[pj]) : 0.0;
        if ((uint32_t)cJ[h] >= (uint32_t)kGT) cJ[h] = -1;
      }
      add_pairs(cI, vI, cJ, vJ, lI);
    }
  }
  __syncthreads();
  double* out = partial + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * (kGT * kGT);
  for (int e = threadIdx.x; e < kGT * kGT; e += kGThreads) out[e] = tile[(e / kGT) * kGS + e % kGT];
}

// B[I0 + a][J0 + b] = sum over chunks (ascending) of the tiles of pair (I, J),
// and B[J0 + b][I0 + a] the same for I < J; a diagonal tile holds the upper
// triangle (a <= b) only.
__global__ void gram_csr_reduce_kernel(int64_t d, int64_t chunks, const double* __restrict__ partial,
                                       double* __restrict__ B) {
  const int nb = (int)((d + kGT - 1) / kGT);
  int I, J;
  pair_of((int)blockIdx.y, nb, I, J);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kGT * kGT) return;
  const int64_t r = (int64_t)I * kGT + e / kGT, c = (int64_t)J * kGT + e % kGT;
  if (r >= d || c >= d) return;
  const int a = e / kGT, b = e % kGT;
  const int es = (I == J && a > b) ? b * kGT + a : e;  // below the diagonal: the mirrored entry
  const double* src = partial + (int64_t)blockIdx.y * chunks * (kGT * kGT) + es;
  double acc = 0.0;
  for (int64_t q = 0; q < chunks; ++q) acc += src[q * (kGT * kGT)];
  B[r * d + c] = acc;
  if (I != J) B[c * d + r] = acc;
}

template <typename T>
hipError_t launch_typed(const void* vals, const int64_t* row_ptr, const int32_t* col_idx, int64_t n, int64_t d,
                        int64_t nnz, double* partial, double* B, hipStream_t s) {
  const int64_t pairs = tile_pairs(d), chunks = row_chunks(n, d);
  const int64_t rows_per_chunk = (n + chunks - 1) / chunks;
  auto kern = gram_csr_kernel<T>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileBytes);
  if (e != hipSuccess) return e;
  kern<<<dim3((unsigned)pairs, (unsigned)chunks), kGThreads, kTileBytes, s>>>(
      static_cast<const T*>(vals), row_ptr, col_idx, n, d, nnz, rows_per_chunk, partial);
  gram_csr_reduce_kernel<<<dim3((kGT * kGT + 255) / 256, (unsigned)pairs), 256, 0, s>>>(d, chunks, partial, B);
  return hipGetLastError();
}

}  // namespace

size_t gram_csr_partial_elems(int64_t n, int64_t d) {
  return (size_t)tile_pairs(d) * (size_t)row_chunks(n, d) * (size_t)(kGT * kGT);
}

hipError_t launch_gram_csr(int dtype, const void* vals, const int64_t* row_ptr, const int32_t* col_idx,
                           int64_t n, int64_t d, int64_t nnz, double* partial, double* B, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  if (n <= 0 || nnz <= 0) return launch_fill_zero(B, sizeof(double) * (size_t)(d * d), s);
  switch (dtype) {
    case 0: return launch_typed<double>(vals, row_ptr, col_idx, n, d, nnz, partial, B, s);
    case 1: return launch_typed<float>(vals, row_ptr, col_idx, n, d, nnz, partial, B, s);
    case 2: return launch_typed<__hip_bfloat16>(vals, row_ptr, col_idx, n, d, nnz, partial, B, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lev
