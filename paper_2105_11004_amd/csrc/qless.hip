// Algorithm 6: exact leverage scores from a Q-less column-pivoted QR of A
// itself (the Gram-Schmidt SPQR that Section 5 adopts), without a sketch.
//
// Q_j = A_K R^{-1} is never formed.  With s_c the remaining norm^2 of column
// c (||a_c||^2 minus the squares of its R entries so far), step j takes the
// unselected column p of largest s_p (ties: lowest index), sets r_jj =
// sqrt(s_p) and, from the column inner products b = A^T a_p (one pass over
// A), r_jc = (b_c - sum_{i<j} r_ip r_ic) / r_jj, then s_c -= r_jc^2.  It
// stops before a step whose r_jj <= zeta r_00 (the rank rule of Section 7)
// or after kmax steps.  The scores are then ||e_i^T A P_k R_k^{-1}||^2 by
// the same Z and pass 2 as the other modes.
//
// Per step: one pass kernel over A writes per-workgroup partial sums of b
// (dense: 16-byte row vectors with the pivot element as weight; CSR: the
// rows that hold column p, found in a first sweep over the column ids), and
// one single-workgroup step kernel sums them in a fixed order, forms row j
// of R, downdates s and picks the next pivot.  Everything stays on the
// device: the host enqueues kmax steps, and the kernels of the steps after
// the stop return at once.  All sums run in a fixed order (FP64), so the
// result is reproducible bit for bit.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_internal.h"

namespace lev {
namespace {

// ctl (int64): [0] steps done (= rank so far), [1] current pivot, [2] stop flag
// dctl (double): [0] r_00, [1] r_jj of the current pivot
constexpr int kPassThreads = 256;
constexpr int kCsrWaves = 8;
constexpr int kStepThreads = 1024;

__device__ __forceinline__ double f64(double x) { return x; }
__device__ __forceinline__ double f64(float x) { return (double)x; }
__device__ __forceinline__ double f64(__hip_bfloat16 x) { return (double)__bfloat162float(x); }

template <typename T>
__device__ __forceinline__ void unpack(const uint4& v, double* out) {
  constexpr int VE = 16 / (int)sizeof(T);
  const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
  for (int i = 0; i < VE; ++i) out[i] = f64(e[i]);
}

// Dense pass: partial[g][c] = sum over the rows i of workgroup g of
// w_i A[i][c], w_i = A[i][p] (squares: A[i][c]^2).  Thread t takes the
// 16-byte vector v = t % nvs of row offset t / nvs (S vectors per thread
// when a row has more than 256 of them), rows strided by rpi.
template <typename T, int S>
__global__ __launch_bounds__(kPassThreads) void qless_pass_dense_kernel(const T* __restrict__ A, int64_t n, int64_t d,
                                                                        int64_t ld, const int64_t* __restrict__ ctl,
                                                                        int squares, int64_t rows_per_group,
                                                                        double* __restrict__ partial) {
  constexpr int VE = 16 / (int)sizeof(T);
  __shared__ double red[kPassThreads * S * VE];
  if (!squares && ctl[2] != 0) return;
  const int64_t p = squares ? 0 : ctl[1];
  const int nv = (int)((d + VE - 1) / VE);
  const int nvs = nv < kPassThreads ? nv : kPassThreads;
  const int rpi = kPassThreads / nvs;
  const int tid = threadIdx.x;
  const int roff = tid / nvs, v = tid % nvs;
  const bool active = roff < rpi;
  double acc[S][VE];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int e = 0; e < VE; ++e) acc[s][e] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_group;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_group);
  if (active) {
    // U rows per round, loaded one round ahead of the products
    constexpr int U = 4;
    uint4 raw[U][S], nraw[U][S];
    double w[U], nw[U];
    auto load_round = [&](int64_t i0, uint4 (&rr)[U][S], double (&ww)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * rpi;
        const bool ok = i < r1;
        const T* row = A + (ok ? i : r0) * ld;
        ww[u] = !ok ? 0.0 : (squares ? 1.0 : f64(row[p]));
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int vi = v + s * kPassThreads;
          rr[u][s] = (ok && vi < nv) ? reinterpret_cast<const uint4*>(row)[vi] : make_uint4(0, 0, 0, 0);
        }
      }
    };
    const int64_t step = (int64_t)U * rpi;
    if (r0 + roff < r1) load_round(r0 + roff, raw, w);
    for (int64_t i0 = r0 + roff; i0 < r1; i0 += step) {
      if (i0 + step < r1) load_round(i0 + step, nraw, nw);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (w[u] == 0.0) continue;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int vi = v + s * kPassThreads;
          double x[VE];
          unpack<T>(raw[u][s], x);
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            const double xe = (vi * VE + e < d) ? x[e] : 0.0;  // the row's padding past d is not A's
            acc[s][e] = fma(squares ? xe : w[u], xe, acc[s][e]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        w[u] = nw[u];
#pragma unroll
        for (int s = 0; s < S; ++s) raw[u][s] = nraw[u][s];
      }
    }
  }
  // sum over the row offsets in a fixed order
  if (active) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int e = 0; e < VE; ++e) red[((roff * S + s) * nvs + v) * VE + e] = acc[s][e];
  }
  __syncthreads();
  for (int q = tid; q < S * nvs * VE; q += kPassThreads) {
    const int s = q / (nvs * VE), rem = q % (nvs * VE);
    const int vv = rem / VE, e = rem % VE;
    const int64_t c = (int64_t)(vv + s * kPassThreads) * VE + e;
    if (c >= d) continue;
    double t = 0.0;
    for (int ro = 0; ro < rpi; ++ro) t += red[((ro * S + s) * nvs + vv) * VE + e];
    partial[(int64_t)blockIdx.x * d + c] = t;
  }
}

// Position of nonzero e among the task's rows: the largest j < nr with
// rps[j] <= e (rps non-decreasing, rps[0] <= e < rps[nr]).
__device__ __forceinline__ int row_of(const int64_t* rps, int nr, int64_t e) {
  int lo = 0, hi = nr;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rps[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// CSR pass: the same partial sums.  A wave takes 64 consecutive rows at a
// time and adds into its own LDS copy of b (deterministic: one row's
// entries are distinct columns, and the rows go in order); the workgroup
// sums its waves' copies in order at the end.  Step mode: a first sweep
// over the column ids finds the rows holding column p and their a_ip, then
// only those rows are read.  Squares mode: every entry adds its square, one
// row of the chunk at a time.
template <typename T>
__global__ __launch_bounds__(64 * kCsrWaves) void qless_pass_csr_kernel(const T* __restrict__ vals,
                                                                        const int64_t* __restrict__ row_ptr,
                                                                        const int32_t* __restrict__ col_idx,
                                                                        int64_t n, int64_t d, int64_t nnz,
                                                                        const int64_t* __restrict__ ctl, int squares,
                                                                        double* __restrict__ partial) {
  extern __shared__ double sm[];
  if (!squares && ctl[2] != 0) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* priv = sm + (size_t)wave * d;
  double* wrow = sm + (size_t)kCsrWaves * d + wave * 64;
  int64_t* rps = reinterpret_cast<int64_t*>(sm + (size_t)kCsrWaves * d + kCsrWaves * 64) + wave * 65;
  for (int64_t c = lane; c < d; c += 64) priv[c] = 0.0;
  const int32_t p = squares ? -1 : (int32_t)ctl[1];
  const int64_t ntask = (n + 63) / 64;
  for (int64_t task = (int64_t)blockIdx.x * kCsrWaves + wave; task < ntask; task += (int64_t)gridDim.x * kCsrWaves) {
    const int64_t r0 = task * 64;
    const int nr = (int)std::min<int64_t>(64, n - r0);
    // row starts, clamped to [0, nnz] and made non-decreasing (a running max)
    int64_t mine = lane <= nr ? std::min<int64_t>(std::max<int64_t>(row_ptr[r0 + lane], 0), nnz) : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t up = __shfl_up(mine, o, 64);
      if (lane >= o) mine = std::max(mine, up);
    }
    rps[lane] = mine;
    int64_t last = std::min<int64_t>(std::max<int64_t>(row_ptr[r0 + nr], 0), nnz);
    last = std::max(last, __shfl(mine, 63, 64));
    if (lane == 0) rps[64] = last;
    __builtin_amdgcn_wave_barrier();
    if (nr < 64 && lane == nr) rps[nr] = last;
    __builtin_amdgcn_wave_barrier();
    const int64_t N0 = rps[0], N1 = rps[nr];
    if (squares) {
      for (int64_t c0 = N0; c0 < N1; c0 += 64) {
        const int64_t e = c0 + lane;
        const bool ok = e < N1;
        const int32_t col = ok ? col_idx[e] : -1;
        const double x = ok ? f64(vals[e]) : 0.0;
        const int j = ok ? row_of(rps, nr, e) : -1;
        const int jlo = row_of(rps, nr, c0), jhi = row_of(rps, nr, std::min<int64_t>(c0 + 63, N1 - 1));
        for (int jj = jlo; jj <= jhi; ++jj) {
          if (j == jj && (uint32_t)col < (uint32_t)d) priv[col] = fma(x, x, priv[col]);
          __builtin_amdgcn_wave_barrier();
        }
      }
      continue;
    }
    wrow[lane] = 0.0;
    __builtin_amdgcn_wave_barrier();
    for (int64_t c0 = N0; c0 < N1; c0 += 64) {
      const int64_t e = c0 + lane;
      if (e < N1 && col_idx[e] == p) wrow[row_of(rps, nr, e)] = f64(vals[e]);
    }
    __builtin_amdgcn_wave_barrier();
    uint64_t live = __ballot(lane < nr && wrow[lane] != 0.0);
    while (live) {
      const int j = __builtin_ctzll(live);
      live &= live - 1;
      const double w = wrow[j];
      const int64_t s = rps[j], e = rps[j + 1];
      for (int64_t c0 = s; c0 < e; c0 += 64) {
        const int64_t q = c0 + lane;
        if (q < e) {
          const int32_t col = col_idx[q];
          if ((uint32_t)col < (uint32_t)d) priv[col] = fma(w, f64(vals[q]), priv[col]);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int64_t c = threadIdx.x; c < d; c += 64 * kCsrWaves) {
    double t = 0.0;
    for (int w = 0; w < kCsrWaves; ++w) t += sm[(size_t)w * d + c];
    partial[(int64_t)blockIdx.x * d + c] = t;
  }
}

// Argmax of s over the unselected columns (ties: lowest index) in one
// workgroup: returns the pivot (or -1) to every thread.
__device__ int pick_pivot(const double* s, const int32_t* sel, int64_t d, double* vbuf, int* ibuf) {
  double best = -1.0;
  int bi = -1;
  for (int64_t c = threadIdx.x; c < d; c += kStepThreads) {
    if (sel[c]) continue;
    const double v = s[c];
    if (v > best || (v == best && (bi < 0 || c < bi))) {
      best = v;
      bi = (int)c;
    }
  }
  vbuf[threadIdx.x] = best;
  ibuf[threadIdx.x] = bi;
  __syncthreads();
  for (int off = kStepThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double vo = vbuf[threadIdx.x + off];
      const int io = ibuf[threadIdx.x + off];
      const double vm = vbuf[threadIdx.x];
      const int im = ibuf[threadIdx.x];
      if (io >= 0 && (im < 0 || vo > vm || (vo == vm && io < im))) {
        vbuf[threadIdx.x] = vo;
        ibuf[threadIdx.x] = io;
      }
    }
    __syncthreads();
  }
  const int r = ibuf[0];
  __syncthreads();
  return r;
}

// bsum[c] = sum over the groups of partial[g][c], in a fixed order: the
// 1024 threads split into 1024 / d slices (d <= 1024) that each sum every
// slices-th group with four independent accumulators, then slice 0 adds
// the slices in order.
__device__ void sum_partials(const double* __restrict__ partial, int groups, int64_t d, double* red,
                             double* bsum) {
  const int slices = (int)(kStepThreads / d);
  const int t = threadIdx.x;
  const int slice = (int)(t / d), c = (int)(t % d);
  if (slice < slices) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int g = slice;
    for (; g + 3 * slices < groups; g += 4 * slices) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += partial[(int64_t)(g + u * slices) * d + c];
    }
    for (; g < groups; g += slices) a[0] += partial[(int64_t)g * d + c];
    red[t] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  __syncthreads();
  if (t < d) {
    double b = 0.0;
    for (int q = 0; q < slices; ++q) b += red[q * d + t];
    bsum[t] = b;
  }
  __syncthreads();
}

// One step after its pass (first: after the norms pass).  b = the sum of
// the partials (fixed order).
__global__ __launch_bounds__(kStepThreads) void qless_step_kernel(int64_t d, int64_t kmax, int groups,
                                                                  const double* __restrict__ partial, double zeta,
                                                                  double* __restrict__ s, int32_t* __restrict__ sel,
                                                                  double* __restrict__ Rrow, int64_t* __restrict__ ctl,
                                                                  double* __restrict__ dctl,
                                                                  int32_t* __restrict__ piv, int first) {
  __shared__ double vbuf[kStepThreads];
  __shared__ int ibuf[kStepThreads];
  __shared__ double bsum[1024];
  if (ctl[2] != 0) return;
  int64_t j = ctl[0];
  sum_partials(partial, groups, d, vbuf, bsum);
  if (first) {
    for (int64_t c = threadIdx.x; c < d; c += kStepThreads) {
      s[c] = bsum[c];
      sel[c] = 0;
    }
    __syncthreads();
  } else {
    const int64_t p = ctl[1];
    const double rjj = dctl[1];
    double* row = Rrow + j * d;
    for (int64_t c = threadIdx.x; c < d; c += kStepThreads) {
      double r = 0.0;
      if (c == p) {
        r = rjj;
      } else if (!sel[c]) {
        double b = bsum[c];
        for (int64_t i = 0; i < j; ++i) b -= Rrow[i * d + p] * Rrow[i * d + c];
        r = b / rjj;
        s[c] -= r * r;
      }
      row[c] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      sel[p] = 1;
      piv[j] = (int32_t)p;
    }
    ++j;
    __syncthreads();
  }
  if (threadIdx.x == 0) ctl[0] = j;
  if (j >= kmax) {
    if (threadIdx.x == 0) ctl[2] = 1;
    return;
  }
  const int np = pick_pivot(s, sel, d, vbuf, ibuf);
  if (threadIdx.x == 0) {
    const double rjj = np >= 0 ? sqrt(fmax(s[np], 0.0)) : 0.0;
    if (j == 0) dctl[0] = rjj;
    if (np < 0 || !(rjj > 0.0) || rjj <= zeta * dctl[0]) {
      ctl[2] = 1;
    } else {
      ctl[1] = np;
      dctl[1] = rjj;
    }
  }
}

// perm = the pivots, then the other columns ascending; R (d x d, pivoted
// order) from the rows; rank.
__global__ __launch_bounds__(kStepThreads) void qless_finalize_kernel(int64_t d, const int64_t* __restrict__ ctl,
                                                                      const int32_t* __restrict__ sel,
                                                                      const int32_t* __restrict__ piv,
                                                                      const double* __restrict__ Rrow,
                                                                      int32_t* __restrict__ perm,
                                                                      double* __restrict__ R,
                                                                      int64_t* __restrict__ rank) {
  __shared__ int32_t pm[1024];
  const int64_t k = ctl[0];
  if (threadIdx.x == 0) {
    int64_t q = 0;
    for (; q < k; ++q) pm[q] = piv[q];
    for (int64_t c = 0; c < d; ++c)
      if (!(c < d && sel[c])) pm[q++] = (int32_t)c;
    *rank = k;
  }
  __syncthreads();
  for (int64_t c = threadIdx.x; c < d; c += kStepThreads) perm[c] = pm[c];
  for (int64_t e = threadIdx.x; e < d * d; e += kStepThreads) {
    const int64_t i = e / d, jp = e % d;
    R[e] = (i < k && jp >= i) ? Rrow[i * d + pm[jp]] : 0.0;
  }
}

template <typename T>
hipError_t pass_dense(const void* A, int64_t n, int64_t d, int64_t ld, const int64_t* ctl, int squares, int groups,
                      double* partial, hipStream_t st) {
  constexpr int VE = 16 / (int)sizeof(T);
  const int64_t nv = (d + VE - 1) / VE;
  const int64_t rows = (n + groups - 1) / groups;
  const T* a = static_cast<const T*>(A);
  if (nv > kPassThreads)
    qless_pass_dense_kernel<T, 2><<<groups, kPassThreads, 0, st>>>(a, n, d, ld, ctl, squares, rows, partial);
  else
    qless_pass_dense_kernel<T, 1><<<groups, kPassThreads, 0, st>>>(a, n, d, ld, ctl, squares, rows, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t pass_csr(const void* vals, const int64_t* row_ptr, const int32_t* col_idx, int64_t n, int64_t d,
                    int64_t nnz, const int64_t* ctl, int squares, int groups, double* partial, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)kCsrWaves * d + kCsrWaves * 64) + sizeof(int64_t) * kCsrWaves * 65;
  auto kern = qless_pass_csr_kernel<T>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  kern<<<groups, 64 * kCsrWaves, lds, st>>>(static_cast<const T*>(vals), row_ptr, col_idx, n, d, nnz, ctl, squares,
                                            partial);
  return hipGetLastError();
}

}  // namespace

int qless_groups(int64_t n, bool csr) {
  const int64_t per = csr ? 64 * kCsrWaves : 256;
  const int64_t cap = csr ? 512 : 1024;  // dense: four workgroups per CU to keep loads in flight
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + per - 1) / per));
}

size_t qless_ws_doubles(int64_t n, int64_t d, int64_t kmax, bool csr) {
  // s, Rrow, partial, dctl (2) and, as doubles, sel, piv and ctl
  return (size_t)d + (size_t)kmax * d + (size_t)qless_groups(n, csr) * d + 2 + (size_t)d + (size_t)kmax + 4;
}

hipError_t launch_qless_qr(const QlessInput& in, int64_t kmax, double zeta, double* ws, int32_t* perm_out,
                           double* R_out, int64_t* rank_out, hipStream_t st) {
  const int64_t n = in.n, d = in.d;
  const bool csr = in.row_ptr != nullptr;
  const int groups = qless_groups(n, csr);
  double* s = ws;
  double* Rrow = s + d;
  double* partial = Rrow + kmax * d;
  double* dctl = partial + (size_t)groups * d;
  int32_t* sel = reinterpret_cast<int32_t*>(dctl + 2);
  int32_t* piv = sel + d;
  int64_t* ctl = reinterpret_cast<int64_t*>(reinterpret_cast<double*>(sel) + d + kmax);
  hipError_t e = launch_fill_zero(ctl, 4 * sizeof(int64_t), st);
  if (e != hipSuccess) return e;
  e = launch_fill_zero(partial, sizeof(double) * (size_t)groups * d, st);
  if (e != hipSuccess) return e;
  auto pass = [&](int squares) -> hipError_t {
    if (n == 0) return hipSuccess;
    if (csr) {
      switch (in.dtype) {
        case 0: return pass_csr<double>(in.values, in.row_ptr, in.col_idx, n, d, in.nnz, ctl, squares, groups, partial, st);
        case 1: return pass_csr<float>(in.values, in.row_ptr, in.col_idx, n, d, in.nnz, ctl, squares, groups, partial, st);
        case 2:
          return pass_csr<__hip_bfloat16>(in.values, in.row_ptr, in.col_idx, n, d, in.nnz, ctl, squares, groups,
                                          partial, st);
        default: return hipErrorInvalidValue;
      }
    }
    switch (in.dtype) {
      case 0: return pass_dense<double>(in.values, n, d, in.ld, ctl, squares, groups, partial, st);
      case 1: return pass_dense<float>(in.values, n, d, in.ld, ctl, squares, groups, partial, st);
      case 2: return pass_dense<__hip_bfloat16>(in.values, n, d, in.ld, ctl, squares, groups, partial, st);
      default: return hipErrorInvalidValue;
    }
  };
  if ((e = pass(1)) != hipSuccess) return e;
  qless_step_kernel<<<1, kStepThreads, 0, st>>>(d, kmax, groups, partial, zeta, s, sel, Rrow, ctl, dctl, piv, 1);
  for (int64_t j = 0; j < kmax; ++j) {
    if ((e = pass(0)) != hipSuccess) return e;
    qless_step_kernel<<<1, kStepThreads, 0, st>>>(d, kmax, groups, partial, zeta, s, sel, Rrow, ctl, dctl, piv, 0);
  }
  qless_finalize_kernel<<<1, kStepThreads, 0, st>>>(d, ctl, sel, piv, Rrow, perm_out, R_out, rank_out);
  return hipGetLastError();
}

}  // namespace lev
