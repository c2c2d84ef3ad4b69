// Helpers of the refined rank-revealing factorisation (Algorithm 4, step 2,
// with the column-pivoted QR of the paper's implementation, Section 7, and
// its cutoff rule |R_kk| < c |R_11| at cutoffs down to the c = 1e-10 of its
// FP64 experiment).
//
// The pivoted Cholesky of the Gram matrix B = A~^T A~ picks the QRCP pivots
// only while the residual column norms stay well above sqrt(u) * R_00: B is
// rounded at u * R_00^2, so below that the Schur diagonal is noise.  The
// refined path therefore runs the Gram pivoting only down to a coarse cutoff
// tau (stage 1, r1 columns), orthonormalises those columns accurately
// (Cholesky QR twice: Q1 with Q1^T Q1 = I to rounding), projects them out of
// the other columns twice (block Gram-Schmidt with reorthogonalisation), and
// pivots again on the Gram of that explicit residual (stage 2, r2 more
// columns), whose rounding is relative to the residual's own norm, not to
// R_00.  The rows of R come from Q^T X (accurate to rounding relative to
// ||X||): R = [Q1^T X; Q2^T X2], Q2 from Cholesky QR twice of the stage-2
// columns.  In exact arithmetic every step equals the corresponding step of
// Householder QRCP (same pivots, same R with positive diagonal), because
// QRCP's trailing matrix after r1 steps has the Gram of the projected
// residual.
//
// The kernels here only move data: the products run on the FP64 GEMM, the
// factorisations on the pivoted Cholesky (pivchol.hip, also in its
// fixed-order mode), the inverses on the blocked solve (trsm.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kMaxD = 1024;

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// X1[i][j] = j < r ? At[i][perm[j]] : 0,  X2[i][j] = j >= r ? At[i][perm[j]] : 0
// (m x d, row-major; X2 may be null).
__global__ void gather_split_kernel(int64_t m, int64_t d, const int32_t* __restrict__ perm,
                                    const int64_t* __restrict__ rank, const double* __restrict__ At,
                                    double* __restrict__ X1, double* __restrict__ X2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  const int64_t i = idx / d, j = idx % d;
  const int64_t r = *rank;
  const double v = At[i * d + perm[j]];
  X1[idx] = j < r ? v : 0.0;
  if (X2 != nullptr) X2[idx] = j < r ? 0.0 : v;
}

// dst += a + b (n elements)
__global__ void add2_kernel(int64_t n, double* __restrict__ dst, const double* __restrict__ a,
                            const double* __restrict__ b) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  dst[idx] += a[idx] + b[idx];
}

// Final permutation, factor and rank from the two rounds.
//  perm1: stage 1 (pivots 0..r1-1, then the other columns); positions of
//         perm1 are the column space of X = A~[:, perm1], Rtop and Rbot.
//  perm2: stage 2 pivots as positions in that space (0..r2-1 valid).
//  perm_out[j]: perm1[j] (j < r1), perm1[perm2[j - r1]] (r1 <= j < r), then
//  the unselected original columns ascending.
//  R_out[j][t] (t >= j): Rtop[j][pos(t)] for j < r1, Rbot[j - r1][pos(t)] for
//  r1 <= j < r, with pos(t) the perm1-position of column perm_out[t]; every
//  other entry zero.  rank_out = r1 + r2.
// One launch: every workgroup rebuilds perm_out and pos in LDS, workgroup 0
// writes perm_out and the rank, each workgroup writes kRows rows of R.
constexpr int kRows = 4;

__global__ __launch_bounds__(kMaxD) void assemble_kernel(int64_t d, const int32_t* __restrict__ perm1,
                                                         const int64_t* __restrict__ rank1,
                                                         const int32_t* __restrict__ perm2,
                                                         const int64_t* __restrict__ rank2,
                                                         const double* __restrict__ Rtop,
                                                         const double* __restrict__ Rbot,
                                                         int32_t* __restrict__ perm_out, double* __restrict__ R_out,
                                                         int64_t* __restrict__ rank_out) {
  __shared__ int chosen[kMaxD];
  __shared__ int inv1[kMaxD];  // original column -> perm1 position
  __shared__ int perm_s[kMaxD];
  __shared__ int wave_cnt[kMaxD / 64];
  const int c = threadIdx.x;
  const int lane = c & 63, w = c >> 6;
  const int r1 = (int)*rank1, r2 = (int)*rank2;
  const int r = r1 + r2;
  if (c < d) {
    chosen[c] = 0;
    inv1[perm1[c]] = c;
  }
  __syncthreads();
  int sel = -1;
  if (c < d && c < r1) sel = perm1[c];
  else if (c < d && c < r) sel = perm1[perm2[c - r1]];
  if (sel >= 0) {
    chosen[sel] = 1;
    perm_s[c] = sel;
  }
  __syncthreads();
  const bool free_c = c < d && chosen[c] == 0;
  const unsigned long long bal = __ballot(free_c);
  if (lane == 0) wave_cnt[w] = __popcll(bal);
  __syncthreads();
  int before = __popcll(bal & ((1ull << lane) - 1ull));
  for (int q = 0; q < w; ++q) before += wave_cnt[q];
  if (free_c) perm_s[r + before] = c;
  __syncthreads();
  if (blockIdx.x == 0) {
    if (c < d) perm_out[c] = perm_s[c];
    if (c == 0) *rank_out = r;
  }
  const int64_t j0 = (int64_t)blockIdx.x * kRows;
  const int64_t j1 = j0 + kRows < d ? j0 + kRows : d;
  for (int64_t j = j0; j < j1; ++j)
    for (int64_t t = c; t < d; t += blockDim.x) {
      double v = 0.0;
      if (t >= j && j < r) {
        const int q = inv1[perm_s[t]];
        v = j < r1 ? Rtop[j * d + q] : Rbot[(j - r1) * d + q];
      }
      R_out[j * d + t] = v;
    }
}

// *flag = (*rank == d) ? 1 : 0 (the refined round is then a no-op).
__global__ void full_rank_flag_kernel(int64_t d, const int64_t* __restrict__ rank, int32_t* __restrict__ flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = (*rank == d) ? 1 : 0;
}

}  // namespace

hipError_t launch_gather_split(int64_t m, int64_t d, const int32_t* perm, const int64_t* rank, const double* At,
                               double* X1, double* X2, hipStream_t s) {
  gather_split_kernel<<<blocks_for(m * d), 256, 0, s>>>(m, d, perm, rank, At, X1, X2);
  return hipGetLastError();
}

hipError_t launch_add2(int64_t n, double* dst, const double* a, const double* b, hipStream_t s) {
  add2_kernel<<<blocks_for(n), 256, 0, s>>>(n, dst, a, b);
  return hipGetLastError();
}

hipError_t launch_rrqr_assemble(int64_t d, const int32_t* perm1, const int64_t* rank1, const int32_t* perm2,
                                const int64_t* rank2, const double* Rtop, const double* Rbot, int32_t* perm_out,
                                double* R_out, int64_t* rank_out, hipStream_t s) {
  if (d <= 0 || d > kMaxD) return hipErrorInvalidValue;
  const unsigned threads = (unsigned)(((d + 63) / 64) * 64);
  assemble_kernel<<<(unsigned)((d + kRows - 1) / kRows), threads, 0, s>>>(d, perm1, rank1, perm2, rank2, Rtop, Rbot,
                                                                         perm_out, R_out, rank_out);
  return hipGetLastError();
}

hipError_t launch_full_rank_flag(int64_t d, const int64_t* rank, int32_t* flag, hipStream_t s) {
  full_rank_flag_kernel<<<1, 64, 0, s>>>(d, rank, flag);
  return hipGetLastError();
}

}  // namespace lev
