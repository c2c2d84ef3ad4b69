// Section 6: the right preconditioner of Algorithm 11 built from the
// sketch's factor, and LSQR on the preconditioned operator A N.
//
// Preconditioner.  The sketch A~ = G S A is factored as A~ P = Q R by the
// rank-revealing step; then
//   QR:  N = P R11^{-1}                       (columns past the rank zero);
//   SVD: N = P V_R Sigma^{-1}, R = U_R Sigma V_R^T the SVD of R, which is the
//        V Sigma^{-1} of the SVD of A~ itself (A~ = (Q U_R) Sigma (P V_R)^T),
//        keeping the k singular values above zeta sigma_1.
// The SVD of R (d <= 128) is the preconditioned one-sided Jacobi method of
// Drmac and Veselic (2008): Hestenes' iteration on W = R^T, whose columns
// are the rows of the pivoted factor and so are already close to
// orthogonal (few sweeps).  W sits in LDS; each round of a round-robin
// ordering orthogonalises all its disjoint column pairs at once (a 16-lane
// group per pair, Rutishauser's rotation), and sweeps repeat until no pair
// is rotated.  Then W = R^T U_R = V_R Sigma: the column norms are the
// singular values and column c over its norm is the right singular vector,
// so N = P W Sigma^{-2} without accumulating the rotations.  Relative
// accuracy of the singular values does not depend on kappa(R).
//
// LSQR (Paige and Saunders 1982) on M = A N from y = 0, with x = N y at the
// end.  Per iteration two passes over A (dense, FP64 arithmetic on any
// storage type) and one single-workgroup kernel:
//   gemv:  t = A (N v) - alpha u, and per-workgroup sums of t_i^2;
//   atv:   beta = sqrt(sum), u = t / beta, per-workgroup partials of A^T u;
//   step:  q = N^T (A^T u) - beta v, alpha = ||q||, v = q / alpha, the
//          rotation (rho, c, s, theta, phi), y += (phi / rho) w,
//          w = v - (theta / rho) w, z = N v for the next gemv.
// Scalars stay in device memory; all sums run in a fixed order.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kSvdGroup = 16;           // lanes per column pair
constexpr int kSvdMaxThreads = 1024;    // 64 groups: every pair of a round at d <= 128
constexpr int kSvdElems = 8;            // column elements per lane at d <= 128
constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum over each 16-lane group, returned to every lane of the group.
__device__ __forceinline__ double group16_sum(double x) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o, 16);
  return x;
}

// Round-robin pairing of dd (even) columns: in round t pair q joins the
// columns at positions q and dd - 1 - q of the ring, where position 0
// holds column 0 for good and position i > 0 holds column
// 1 + (i - 1 + t) mod (dd - 1); so from one round to the next every
// column but 0 moves to the next of 1 .. dd - 1, cyclically.
__device__ __forceinline__ int rr_col(int dd, int t, int i) { return i == 0 ? 0 : 1 + (i - 1 + t) % (dd - 1); }
__device__ __forceinline__ int rr_next(int dd, int c) { return c == 0 ? 0 : (c + 1 == dd ? 1 : c + 1); }

// v + v of the DPP partner lane (both 32-bit halves moved).
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}

// Sum over each 16-lane row by butterflies whose partners always sit in
// the other half of the part summed so far, so both sides add the same two
// values and every lane of the row ends with identical bits (the rotation
// is then the same in every lane).  All 16 lanes must be active.
__device__ __forceinline__ double row16_sum(double v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v = dpp_add<0x141>(v);  // row_half_mirror
  v = dpp_add<0x140>(v);  // row_mirror
  return v;
}

// One workgroup of 16 * (dd / 2) lanes (rounded up to a wave); LDS holds W
// column-major, dd columns of d (a zero column pads an odd d).
__global__ __launch_bounds__(kSvdMaxThreads) void jacobi_svd_kernel(int64_t d, const double* __restrict__ R,
                                                                    const int64_t* __restrict__ rank,
                                                                    const int32_t* __restrict__ perm, double zeta,
                                                                    double* __restrict__ N,
                                                                    int64_t* __restrict__ k_out) {
  extern __shared__ double W[];
  __shared__ int rotated;
  __shared__ double sig[128];
  __shared__ int order[128];
  const int di = (int)d;
  const int dd = di + (di & 1);
  const int64_t r = *rank;
  // column c of W = row c of R (rows past the rank are zero)
  for (int e = threadIdx.x; e < dd * di; e += blockDim.x) {
    const int c = e / di, i = e - c * di;
    W[e] = (c < di && c < r) ? R[(int64_t)c * d + i] : 0.0;
  }
  __syncthreads();
  const int gl = threadIdx.x & (kSvdGroup - 1);
  const int q = threadIdx.x / kSvdGroup;
  const bool active = q < dd / 2;  // whole 16-lane rows are active or not
  // a pair is rotated while |x . y| > tol ||x|| ||y||, tested squared
  const double tol = 4.0 * (double)di * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    int a = rr_col(dd, 0, q), b = rr_col(dd, 0, dd - 1 - q);
    for (int t = 0; t < dd - 1; ++t, a = rr_next(dd, a), b = rr_next(dd, b)) {
      if (active) {
        double* wa = W + a * di;
        double* wb = W + b * di;
        double x[kSvdElems], y[kSvdElems];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int j = 0; j < kSvdElems; ++j) {
          // the load's index is clamped into the column and its value
          // zeroed after, so no load sits under a branch
          const int i = gl + kSvdGroup * j;
          const int ic = i < di ? i : di - 1;
          x[j] = i < di ? wa[ic] : 0.0;
          y[j] = i < di ? wb[ic] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kSvdElems; ++j) {
          al = fma(x[j], x[j], al);
          be = fma(y[j], y[j], be);
          ga = fma(x[j], y[j], ga);
        }
        al = row16_sum(al);
        be = row16_sum(be);
        ga = row16_sum(ga);
        if (ga != 0.0 && ga * ga > tol2 * (al * be)) {
          const double zt = (be - al) / (2.0 * ga);
          const double tn = (zt >= 0.0 ? 1.0 : -1.0) / (fabs(zt) + sqrt(1.0 + zt * zt));
          const double c = rsqrt(1.0 + tn * tn), s = c * tn;  // 1 + tn^2 in [1, 2]
#pragma unroll
          for (int j = 0; j < kSvdElems; ++j) {
            const int i = gl + kSvdGroup * j;
            if (i < di) {
              wa[i] = c * x[j] - s * y[j];
              wb[i] = s * x[j] + c * y[j];
            }
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // singular values, their descending order (ties: lower column first), k
  for (int c = threadIdx.x; c < di; c += blockDim.x) {
    double nn = 0.0;
    for (int i = 0; i < di; ++i) nn = fma(W[c * di + i], W[c * di + i], nn);
    sig[c] = sqrt(nn);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < di; c += blockDim.x) {
    int rk = 0;
    for (int c2 = 0; c2 < di; ++c2) rk += (sig[c2] > sig[c] || (sig[c2] == sig[c] && c2 < c)) ? 1 : 0;
    order[rk] = c;
  }
  __syncthreads();
  const double s1 = sig[order[0]];
  int k = 0;
  for (int c = 0; c < di; ++c) k += (s1 > 0.0 && sig[order[c]] > zeta * s1) ? 1 : 0;
  // N[perm[i]][c] = V_R[i][order[c]] / sigma = W[i][order[c]] / sigma^2
  for (int e = threadIdx.x; e < di * di; e += blockDim.x) {
    const int i = e / di, c = e - i * di;
    double v = 0.0;
    if (c < k) {
      const int o = order[c];
      v = W[o * di + i] / sig[o] / sig[o];
    }
    N[(int64_t)perm[i] * d + c] = v;
  }
  if (threadIdx.x == 0) *k_out = k;
}

// N[perm[j]][q] = Z[j][q] (Z = R11^{-1} with zero rows past the rank).
__global__ void scatter_rows_kernel(int64_t d, const int32_t* __restrict__ perm, const double* __restrict__ Z,
                                    double* __restrict__ N, const int64_t* __restrict__ rank,
                                    int64_t* __restrict__ k_out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *k_out = *rank;
  if (e >= d * d) return;
  const int64_t j = e / d, q = e % d;
  N[(int64_t)perm[j] * d + q] = Z[e];
}

// ---- LSQR -------------------------------------------------------------------------
// st: [0] alpha, [1] beta, [2] rhobar, [3] phibar, [4] stop (0 / 1), [5] beta_1
constexpr int kGemvThreads = 256;
constexpr int kStepThreads = 1024;

__device__ __forceinline__ double f64(double x) { return x; }
__device__ __forceinline__ double f64(float x) { return (double)x; }
__device__ __forceinline__ double f64(__hip_bfloat16 x) { return (double)__bfloat162float(x); }

// Four consecutive elements of a row from column c (c a multiple of 4,
// c < d), widened to FP64; elements at or past d read as zero.  Rows are
// 16-byte aligned with ld * sizeof(T) a multiple of 16, so a vector whose
// first element is below d stays inside the row (FP64: each 16-byte half
// is read only when its first element is below d).
__device__ __forceinline__ void load4(const float* p, int64_t c, int64_t d, double (&a)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a[0] = v.x;
  a[1] = c + 1 < d ? (double)v.y : 0.0;
  a[2] = c + 2 < d ? (double)v.z : 0.0;
  a[3] = c + 3 < d ? (double)v.w : 0.0;
}
__device__ __forceinline__ void load4(const double* p, int64_t c, int64_t d, double (&a)[4]) {
  const double2 lo = *reinterpret_cast<const double2*>(p);
  const double2 hi = c + 2 < d ? *reinterpret_cast<const double2*>(p + 2) : make_double2(0.0, 0.0);
  a[0] = lo.x;
  a[1] = c + 1 < d ? lo.y : 0.0;
  a[2] = hi.x;
  a[3] = c + 3 < d ? hi.y : 0.0;
}
__device__ __forceinline__ void load4(const __hip_bfloat16* p, int64_t c, int64_t d, double (&a)[4]) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  a[0] = (double)__uint_as_float(v.x << 16);
  a[1] = c + 1 < d ? (double)__uint_as_float(v.x & 0xFFFF0000u) : 0.0;
  a[2] = c + 2 < d ? (double)__uint_as_float(v.y << 16) : 0.0;
  a[3] = c + 3 < d ? (double)__uint_as_float(v.y & 0xFFFF0000u) : 0.0;
}

// t_i = A[i,:] z - alpha u_i (or b_i when init), partial[g] = sum of t_i^2
// over the workgroup's rows.  A 16-lane group takes a row: lane l of the
// group reads elements 64 m + 4 l .. + 3 (one vector load per 64 columns,
// four rows per wave-instruction, each 256 contiguous bytes), z comes from
// LDS, and the row's sum is a four-step reduction over the group; two rows
// per group are in flight at a time.
constexpr int kGemvGroup = 16;
template <typename T>
__global__ __launch_bounds__(kGemvThreads) void lsqr_gemv_kernel(const T* __restrict__ A, int64_t n, int64_t d,
                                                                 int64_t ld, const double* __restrict__ z,
                                                                 const double* __restrict__ u,
                                                                 const double* __restrict__ b, int init,
                                                                 const double* __restrict__ st,
                                                                 double* __restrict__ t, double* __restrict__ partial) {
  __shared__ double red[kGemvThreads / 64];
  __shared__ __align__(16) double zs[1024 + 4];
  if (!init && st[4] != 0.0) return;
  const double alpha = init ? 0.0 : st[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane % kGemvGroup;
  const int row_slot = threadIdx.x / kGemvGroup;  // 0 .. 15 in the workgroup
  constexpr int kSlots = kGemvThreads / kGemvGroup;
  const int64_t rows_per_group = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_group, r1 = std::min<int64_t>(n, r0 + rows_per_group);
  if (!init)
    for (int64_t c = threadIdx.x; c < d; c += kGemvThreads) zs[c] = z[c];
  __syncthreads();
  const int nm = (int)((d + 63) / 64);
  auto row_dot = [&](int64_t i) -> double {
    double acc = 0.0;
    for (int m = 0; m < nm; ++m) {
      const int64_t c = 64 * m + 4 * gl;
      if (c < d) {
        double a[4];
        load4(A + i * ld + c, c, d, a);
        const double2 z0 = *reinterpret_cast<const double2*>(zs + c);
        const double2 z1 = *reinterpret_cast<const double2*>(zs + c + 2);
        acc = fma(a[0], z0.x, acc);
        acc = fma(a[1], z0.y, acc);
        acc = fma(a[2], c + 2 < d ? z1.x : 0.0, acc);
        acc = fma(a[3], c + 3 < d ? z1.y : 0.0, acc);
      }
    }
    return acc;
  };
  double sq = 0.0;
  for (int64_t i0 = r0; i0 < r1; i0 += 2 * kSlots) {
    const int64_t ia = i0 + row_slot, ib = ia + kSlots;
    double sa = 0.0, sb = 0.0;
    if (!init) {
      if (ia < r1) sa = row_dot(ia);
      if (ib < r1) sb = row_dot(ib);
      // sum over the 16 lanes of the group (lane 15 of each 16-lane row ends with it)
      sa = group16_sum(sa);
      sb = group16_sum(sb);
    }
    if (gl == kGemvGroup - 1) {
      if (ia < r1) {
        const double ti = init ? b[ia] : sa - alpha * u[ia];
        t[ia] = ti;
        sq = fma(ti, ti, sq);
      }
      if (ib < r1) {
        const double ti = init ? b[ib] : sb - alpha * u[ib];
        t[ib] = ti;
        sq = fma(ti, ti, sq);
      }
    }
  }
  sq = wave_sum(sq);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kGemvThreads / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// beta = sqrt(sum of the gemv partials); u = t / beta; partial_g[c] = sum over
// the workgroup's rows of u_i A[i][c].  Per 256-column slice, lane l of a
// wave takes columns 4 l .. 4 l + 3 (one vector load per row), the four
// waves take every fourth row with eight rows in flight per lane, and the
// waves' sums are added in LDS in wave order (fixed: deterministic bits).
constexpr int kAtvCols = 256;
constexpr int kAtvRows = 8;
template <typename T>
__global__ __launch_bounds__(kGemvThreads) void lsqr_atv_kernel(const T* __restrict__ A, int64_t n, int64_t d,
                                                                int64_t ld, const double* __restrict__ t,
                                                                const double* __restrict__ gpart, int ggroups,
                                                                double* __restrict__ st, int init,
                                                                double* __restrict__ u, double* __restrict__ partial) {
  __shared__ double red[kGemvThreads / 64][kAtvCols];
  if (!init && st[4] != 0.0) return;
  double s = 0.0;
  for (int g = 0; g < ggroups; ++g) s += gpart[g];
  const double beta = sqrt(s);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[1] = beta;
    if (init) {
      st[5] = beta;
      st[3] = beta;  // phibar = beta_1
    }
  }
  const int64_t rows_per_group = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_group, r1 = std::min<int64_t>(n, r0 + rows_per_group);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += kGemvThreads) u[i] = t[i] * inv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kW = kGemvThreads / 64;
  for (int64_t c0 = 0; c0 < d; c0 += kAtvCols) {
    const int64_t c = c0 + 4 * lane;
    const bool live = c < d;
    const int64_t cl = live ? c : 0;  // lanes past d read column 0 and add nothing
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = r0 + wave;
    for (; i + kW * (kAtvRows - 1) < r1; i += kW * kAtvRows) {
      double a[kAtvRows][4];
      double ui[kAtvRows];
#pragma unroll
      for (int q = 0; q < kAtvRows; ++q) {
        load4(A + (i + kW * q) * ld + cl, cl, d, a[q]);
        ui[q] = live ? t[i + kW * q] * inv : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kAtvRows; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fma(ui[q], a[q][e], acc[e]);
    }
    for (; i < r1; i += kW) {
      double a[4];
      load4(A + i * ld + cl, cl, d, a);
      const double ui = live ? t[i] * inv : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = fma(ui, a[e], acc[e]);
    }
    __syncthreads();  // the previous slice's sums have been read
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave][4 * lane + e] = acc[e];
    __syncthreads();
    const int64_t cc = c0 + threadIdx.x;
    if (threadIdx.x < kAtvCols && cc < d) {
      double v = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kW; ++w) v += red[w][threadIdx.x];
      partial[(int64_t)blockIdx.x * d + cc] = v;
    }
  }
}

// One LSQR step after the two passes (init: the first alpha, v, w).
__global__ __launch_bounds__(kStepThreads) void lsqr_step_kernel(int64_t d, const double* __restrict__ N,
                                                                 const double* __restrict__ partial, int groups,
                                                                 double* __restrict__ st, double* __restrict__ v,
                                                                 double* __restrict__ w, double* __restrict__ y,
                                                                 double* __restrict__ z, double* __restrict__ hist,
                                                                 int64_t it, int init) {
  __shared__ double g[1024];
  __shared__ double q[1024];
  __shared__ double red[kStepThreads / 64];
  if (!init && st[4] != 0.0) {
    if (threadIdx.x == 0 && hist != nullptr) hist[it] = st[3];
    return;
  }
  const int di = (int)d;
  // g = the sum of the workgroups' partials (eight independent partial sums
  // per column, so that eight loads are in flight, added in a fixed order)
  constexpr int kU = 8;
  for (int c = threadIdx.x; c < di; c += kStepThreads) {
    double sp[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) sp[u] = 0.0;
    int gg = 0;
    for (; gg + kU <= groups; gg += kU)
#pragma unroll
      for (int u = 0; u < kU; ++u) sp[u] += partial[(int64_t)(gg + u) * d + c];
    for (; gg < groups; ++gg) sp[0] += partial[(int64_t)gg * d + c];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u) s += sp[u];
    g[c] = s;
  }
  __syncthreads();
  const double beta = st[1];
  // q = N^T g - beta v
  double sq = 0.0;
  for (int c = threadIdx.x; c < di; c += kStepThreads) {
    double sp[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) sp[u] = 0.0;
    int i = 0;
    for (; i + kU <= di; i += kU)
#pragma unroll
      for (int u = 0; u < kU; ++u) sp[u] = fma(N[(int64_t)(i + u) * d + c], g[i + u], sp[u]);
    for (; i < di; ++i) sp[0] = fma(N[(int64_t)i * d + c], g[i], sp[0]);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u) s += sp[u];
    const double qc = init ? s : s - beta * v[c];
    q[c] = qc;
    sq = fma(qc, qc, sq);
  }
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  double a2 = 0.0;
  for (int wv = 0; wv < kStepThreads / 64; ++wv) a2 += red[wv];
  const double alpha = sqrt(a2);
  const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
  double rho = 1.0, c = 1.0, s = 0.0, phi = 0.0;
  const double rhobar = st[2], phibar = st[3];
  if (!init) {
    rho = hypot(rhobar, beta);
    c = rhobar / rho;
    s = beta / rho;
  }
  const double theta = s * alpha;
  phi = c * phibar;
  for (int cc = threadIdx.x; cc < di; cc += kStepThreads) {
    const double vn = q[cc] * ia;
    if (init) {
      w[cc] = vn;
      y[cc] = 0.0;
    } else {
      y[cc] = fma(phi / rho, w[cc], y[cc]);
      w[cc] = vn - (theta / rho) * w[cc];
    }
    v[cc] = vn;
    g[cc] = vn;  // (g is free again: v in LDS for z below)
  }
  __syncthreads();
  // z = N v for the next gemv: a wave per row, its lanes along the row
  // (coalesced), then a wave sum
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = wv; r < di; r += kStepThreads / 64) {
      double acc = 0.0;
      for (int cc = lane; cc < di; cc += 64) acc = fma(N[(int64_t)r * d + cc], g[cc], acc);
      acc = wave_sum(acc);
      if (lane == 0) z[r] = acc;
    }
  }
  if (threadIdx.x == 0) {
    st[0] = alpha;
    if (init) {
      st[2] = alpha;  // rhobar = alpha_1
    } else {
      st[2] = -c * alpha;
      st[3] = s * phibar;
      if (hist != nullptr) hist[it] = s * phibar;
    }
    if (alpha == 0.0 || (!init && beta == 0.0) || st[5] == 0.0) st[4] = 1.0;
  }
}

// x = N y.
__global__ void lsqr_finish_kernel(int64_t d, const double* __restrict__ N, const double* __restrict__ y,
                                   double* __restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d) return;
  double acc = 0.0;
  for (int64_t c = 0; c < d; ++c) acc = fma(N[r * d + c], y[c], acc);
  x[r] = acc;
}

template <typename T>
hipError_t lsqr_typed(const void* Av, int64_t n, int64_t d, int64_t ld, const double* N, const double* b,
                      int64_t iters, double* x, double* hist, double* ws, hipStream_t s) {
  const T* A = static_cast<const T*>(Av);
  const int groups = lsqr_groups(n);
  double* st = ws;               // 8
  double* u = st + 8;            // n
  double* t = u + n;             // n
  double* gpart = t + n;         // groups
  double* apart = gpart + groups;  // groups * d
  double* v = apart + (size_t)groups * d;  // d
  double* w = v + d;
  double* y = w + d;
  double* z = y + d;
  hipError_t e = launch_fill_zero(st, 8 * sizeof(double), s);
  if (e != hipSuccess) return e;
  // beta_1 u_1 = b; alpha_1 v_1 = M^T u_1
  lsqr_gemv_kernel<T><<<groups, kGemvThreads, 0, s>>>(A, n, d, ld, z, u, b, 1, st, t, gpart);
  lsqr_atv_kernel<T><<<groups, kGemvThreads, 0, s>>>(A, n, d, ld, t, gpart, groups, st, 1, u, apart);
  lsqr_step_kernel<<<1, kStepThreads, 0, s>>>(d, N, apart, groups, st, v, w, y, z, hist, 0, 1);
  for (int64_t it = 0; it < iters; ++it) {
    lsqr_gemv_kernel<T><<<groups, kGemvThreads, 0, s>>>(A, n, d, ld, z, u, b, 0, st, t, gpart);
    lsqr_atv_kernel<T><<<groups, kGemvThreads, 0, s>>>(A, n, d, ld, t, gpart, groups, st, 0, u, apart);
    lsqr_step_kernel<<<1, kStepThreads, 0, s>>>(d, N, apart, groups, st, v, w, y, z, hist, it, 0);
  }
  lsqr_finish_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, N, y, x);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_precondition(int method, int64_t d, const double* R, const int64_t* rank, const int32_t* perm,
                               double zeta, double* work, double* N, int64_t* k_out, int32_t* err,
                               hipStream_t s) {
  if (method == 1) {
    if (d > 128) return hipErrorInvalidValue;
    const int64_t dd = d + (d & 1);
    const size_t lds = sizeof(double) * (size_t)(dd * d);  // <= 128 KiB
    const int threads = (int)std::max<int64_t>(64, (dd / 2 * kSvdGroup + 63) / 64 * 64);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(jacobi_svd_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    jacobi_svd_kernel<<<1, threads, lds, s>>>(d, R, rank, perm, zeta, N, k_out);
    return hipGetLastError();
  }
  // QR: Z = R11^{-1} (trsm of the identity), rows scattered to the original columns
  double* I = work;
  double* Z = work + d * d;
  hipError_t e = launch_identity(d, I, s);
  if (e != hipSuccess) return e;
  e = launch_trsm_z(d, d, R, rank, I, Z, err, s);
  if (e != hipSuccess) return e;
  scatter_rows_kernel<<<(unsigned)((d * d + 255) / 256), 256, 0, s>>>(d, perm, Z, N, rank, k_out);
  return hipGetLastError();
}

// k = -1 when a bounded wait of the rank-revealing step ran out.
__global__ void flag_error_kernel(const int32_t* __restrict__ err, int64_t* __restrict__ k_out) {
  if (*err != 0) *k_out = -1;
}

hipError_t launch_flag_error(const int32_t* err, int64_t* k_out, hipStream_t s) {
  flag_error_kernel<<<1, 1, 0, s>>>(err, k_out);
  return hipGetLastError();
}

int lsqr_groups(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256)); }

size_t lsqr_ws_doubles(int64_t n, int64_t d) {
  return 8 + 2 * (size_t)n + (size_t)lsqr_groups(n) * (1 + (size_t)d) + 4 * (size_t)d;
}

hipError_t launch_lsqr(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, const double* N, const double* b,
                       int64_t iters, double* x, double* hist, double* ws, hipStream_t s) {
  switch (dtype) {
    case 0: return lsqr_typed<double>(A, n, d, ld, N, b, iters, x, hist, ws, s);
    case 1: return lsqr_typed<float>(A, n, d, ld, N, b, iters, x, hist, ws, s);
    case 2: return lsqr_typed<__hip_bfloat16>(A, n, d, ld, N, b, iters, x, hist, ws, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lev
