// Rank-revealing factorisation of the sketch (Algorithm 4, step 2, with the
// classical column-pivoted QR that the paper's implementation uses in place
// of the strong RRQR, Section 7).
//
// Column-pivoted QR of A~ chooses, at step J, the remaining column with the
// largest residual norm after projecting out the J columns already chosen.
// Those residual norms^2 are exactly the diagonal of the Schur complement of
// the Gram matrix B = A~^T A~ after J steps of symmetric pivoted Cholesky,
// and the Cholesky factor is the QR factor with positive diagonal.  On the
// GPU the Cholesky form is the cheap one: one pivot step needs only the
// pivot's row of the current Schur complement, O(d * nb) work that one
// workgroup does in registers, where Householder QRCP needs a pass over the
// whole trailing matrix per pivot.  Pivoting is blocked in panels of NB
// steps (one workgroup, thread c owns column c) followed by a rank-NB
// update of the Schur complement on the matrix cores (dgemm).
//
// Rank rule (the cutoff test of Section 7): pivoting stops at the first J
// with R_JJ <= zeta * R_00 (or a non-positive Schur diagonal); r = J.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr int NB = 32;
constexpr int kMaxD = 1024;

struct ArgMax {
  double v;
  int i;
};

__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b) {
  // larger value wins; ties to the lower column index
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ __forceinline__ ArgMax wave_argmax(ArgMax x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ArgMax o;
    o.v = __shfl_xor(x.v, off);
    o.i = __shfl_xor(x.i, off);
    x = better(x, o);
  }
  return x;
}

// flags[0] = done, flags[1] = pivots computed so far.
__global__ __launch_bounds__(kMaxD) void pivchol_panel_kernel(const double* __restrict__ S, int64_t d,
                                                              double zeta, int64_t J0,
                                                              PivCholState st,
                                                              int64_t* __restrict__ rank_out) {
  __shared__ double bc[NB];
  __shared__ double wv[2][kMaxD / 64];
  __shared__ int wi[2][kMaxD / 64];

  const int c = threadIdx.x;
  const int lane = c & 63, wave = c >> 6;
  const int nwaves = blockDim.x >> 6;
  if (J0 > 0 && st.flags[0] != 0) return;

  double dg;
  if (c < d) dg = (J0 == 0) ? S[(int64_t)c * d + c] : st.diag[c];
  else dg = -INFINITY;
  bool alive = (c < d) && (dg != -INFINITY);
  double r00 = (J0 == 0) ? 0.0 : *st.r00;

  double rp[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) rp[t] = 0.0;

  int64_t J = J0;
  bool stop = false;
  bool active = true;  // uniform across the workgroup
  // Constant trip count (no break) so the loop unrolls fully and rp[] stays
  // in registers.
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (active && J >= d) active = false;
    if (!active) continue;
    ArgMax mine{alive ? dg : -INFINITY, alive ? c : 0x7fffffff};
    mine = wave_argmax(mine);
    if (lane == 0) {
      wv[j & 1][wave] = mine.v;
      wi[j & 1][wave] = mine.i;
    }
    __syncthreads();
    ArgMax best{-INFINITY, 0x7fffffff};
    for (int w = 0; w < nwaves; ++w) best = better(best, ArgMax{wv[j & 1][w], wi[j & 1][w]});
    const double pv = best.v;
    const int p = best.i;
    if (J == 0) r00 = pv > 0.0 ? sqrt(pv) : 0.0;
    if (!(pv > 0.0) || !(sqrt(pv) > zeta * r00)) {
      stop = true;
      active = false;
      continue;
    }
    const double rjj = sqrt(pv);
    // prefetch the pivot row of the Schur complement (symmetric: = column p)
    const double s_pc = (c < d) ? S[(int64_t)p * d + c] : 0.0;
    if (c == p) {
#pragma unroll
      for (int t = 0; t < j; ++t) bc[t] = rp[t];
    }
    __syncthreads();
    double val = 0.0;
    if (c == p) {
      val = rjj;
      alive = false;
      dg = -INFINITY;
    } else if (alive) {
      double acc = s_pc;
#pragma unroll
      for (int t = 0; t < j; ++t) acc = fma(-bc[t], rp[t], acc);
      val = acc / rjj;
      dg = fma(-val, val, dg);
    }
    rp[j] = val;
    if (c < d) st.Rrows[J * d + c] = val;
    if (c == 0) st.piv[J] = p;
    ++J;
  }

  if (c < d) st.diag[c] = dg;
  if (c == 0) {
    *st.r00 = r00;
    st.flags[1] = (int32_t)J;
    if (stop || J >= d) {
      st.flags[0] = 1;
      *rank_out = J;
    }
  }
}

// perm: pivots, then the unselected columns ascending.  R_out: pivoted,
// upper triangular, rows >= r zero.  One workgroup of kMaxD threads for the
// permutation, then the R gather.
__global__ __launch_bounds__(kMaxD) void pivchol_perm_kernel(int64_t d, PivCholState st,
                                                             const int64_t* __restrict__ rank,
                                                             int32_t* __restrict__ perm_out) {
  __shared__ int chosen[kMaxD];
  __shared__ int scan[kMaxD];
  const int c = threadIdx.x;
  const int64_t r = *rank;
  if (c < d) chosen[c] = 0;
  __syncthreads();
  if (c < r) chosen[st.piv[c]] = 1;
  __syncthreads();
  const int free_c = (c < d && !chosen[c]) ? 1 : 0;
  scan[c] = free_c;
  __syncthreads();
  // inclusive Hillis-Steele scan over kMaxD entries
  for (int off = 1; off < kMaxD; off <<= 1) {
    const int add = (c >= off) ? scan[c - off] : 0;
    __syncthreads();
    scan[c] += add;
    __syncthreads();
  }
  if (c < r) perm_out[c] = st.piv[c];
  if (free_c) perm_out[r + scan[c] - 1] = c;
}

__global__ void pivchol_gather_r_kernel(int64_t d, PivCholState st, const int64_t* __restrict__ rank,
                                        const int32_t* __restrict__ perm, double* __restrict__ R_out) {
  const int64_t j = blockIdx.x;  // output row
  const int64_t r = *rank;
  for (int64_t t = threadIdx.x; t < d; t += blockDim.x) {
    double v = 0.0;
    if (j < r && t >= j) v = st.Rrows[j * d + perm[t]];
    R_out[j * d + t] = v;
  }
}

}  // namespace

hipError_t launch_pivchol(double* B, int64_t d, double zeta, const PivCholState& st, int64_t* rank_out,
                          double* gemm_partial, hipStream_t s) {
  (void)gemm_partial;
  if (d <= 0 || d > kMaxD) return hipErrorInvalidValue;
  const int threads = (int)(((d + 63) / 64) * 64);
  for (int64_t J0 = 0; J0 < d; J0 += NB) {
    pivchol_panel_kernel<<<1, threads, 0, s>>>(B, d, zeta, J0, st, rank_out);
    if (J0 + NB < d) {
      // S <- S - R_panel^T R_panel over the panel's NB rows (skipped once done)
      const double* Rp = st.Rrows + J0 * d;
      hipError_t e = launch_dgemm(d, d, NB, -1.0, Rp, 1, d, Rp, d, 1, 1.0, B, d, 1, nullptr,
                                  st.flags, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_pivchol_finalize(int64_t d, const PivCholState& st, const int64_t* rank,
                                   int32_t* perm_out, double* R_out, hipStream_t s) {
  pivchol_perm_kernel<<<1, kMaxD, 0, s>>>(d, st, rank, perm_out);
  pivchol_gather_r_kernel<<<(unsigned)d, 256, 0, s>>>(d, st, rank, perm_out, R_out);
  return hipGetLastError();
}

}  // namespace lev
