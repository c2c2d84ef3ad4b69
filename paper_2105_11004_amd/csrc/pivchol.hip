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
//
// Two implementations: d <= 256 runs entirely in one workgroup with the
// Schur complement in registers (below); larger d uses panels of NB pivots
// (one workgroup) and rank-NB Schur updates on the matrix cores.
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

// ---------------------------------------------------------------------------
// d <= 256: the whole factorisation in one workgroup with the symmetric
// Schur complement resident in registers (right-looking pivoted Cholesky).
//
// The d x d matrix is tiled by 64 x 64 squares that cover its lower triangle
// (10 for d = 256); "square" wave w owns square (a, b) and lane l of that wave
// holds row 64a + l, columns 64b .. 64b + 63 in 128 registers.  Two more
// "diagonal" waves own the Schur diagonal: lane l of diagonal wave q holds
// d_i for rows i = 128 q + l and 128 q + 64 + l, updated as d_i -= l_i^2.
// Twelve waves (three per SIMD) leave up to 170 registers per lane.
//
// Per pivot step (two barriers): every wave reads the per-diagonal-wave
// candidates (value, index) left by the previous step and takes the best, p,
// with 1/sqrt(S_pp) from the hardware estimate plus two Newton steps; the
// owners of column p (rows i >= p) and of row p (columns j < p) publish
// l = S[:, p] / sqrt(S_pp) to LDS; after the barrier the square waves apply
// S -= l l^T to their entries while the diagonal waves, at the same time,
// update d, store R[J, :] = l and leave their argmax (DPP wave reduction) for
// the next step.  No global memory is read inside the loop.
constexpr int kSmallD = 256;
constexpr int kBandR = 64, kBandC = 64;
constexpr int kLvec = 256;  // >= 64 * ceil(256 / 64)

__host__ __device__ inline int small_bands(int a, int d) {
  const int by_tri = (kBandR * a + kBandR - 1) / kBandC + 1;
  const int by_d = (d + kBandC - 1) / kBandC;
  return by_tri < by_d ? by_tri : by_d;
}

__host__ __device__ inline int small_rects(int d) {
  int cnt = 0;
  for (int a = 0; a * kBandR < d; ++a) cnt += small_bands(a, d);
  return cnt;
}

__device__ inline void small_rect(int w, int d, int& a_out, int& b_out) {
  int idx = 0;
  for (int a = 0; a * kBandR < d; ++a) {
    const int nb = small_bands(a, d);
    if (w < idx + nb) {
      a_out = a;
      b_out = w - idx;
      return;
    }
    idx += nb;
  }
  a_out = 0;
  b_out = 0;
}

typedef double v16d __attribute__((ext_vector_type(16)));

// One DPP step of a wave max over doubles (identity -inf).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_max_step(double v) {
  const int olo = 0, ohi = (int)0xFFF00000;  // -inf
  const int slo = __builtin_amdgcn_update_dpp(olo, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int shi = __builtin_amdgcn_update_dpp(ohi, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return fmax(v, __hiloint2double(shi, slo));
}

// Max over the 64 lanes (row shifts within 16-lane rows, then row broadcasts;
// lane 63 ends with the total), returned to every lane.
__device__ __forceinline__ double wave_max_f64(double v) {
  v = dpp_max_step<0x111, 0xF>(v);  // row_shr:1
  v = dpp_max_step<0x112, 0xF>(v);  // row_shr:2
  v = dpp_max_step<0x114, 0xF>(v);  // row_shr:4
  v = dpp_max_step<0x118, 0xF>(v);  // row_shr:8
  v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15
  v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// waits for every outstanding global store to be acknowledged; inside the
// pivot loop the waves exchange data through LDS alone, and the R rows they
// store to global memory are not read back before the kernel ends.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

struct Cand {
  double v;
  int idx;
};
constexpr int kDiagRows = 128;  // rows per diagonal wave (two per lane)

__host__ __device__ inline int small_diag_waves(int d) { return (d + kDiagRows - 1) / kDiagRows; }

__global__ __launch_bounds__(768) void pivchol_small_kernel(const double* __restrict__ B, int d, double zeta,
                                                            PivCholState st, int64_t* __restrict__ rank_out) {
  __shared__ __align__(16) double lvec[kLvec];
  __shared__ Cand cand[kSmallD / kDiagRows];

  const int lane = threadIdx.x & 63;
  // wave-uniform values kept scalar (the compiler cannot infer it)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nrect = small_rects(d);
  const bool square = wave < nrect;  // uniform
  const int ndiag = small_diag_waves(d);
  int a = 0, b = 0;
  if (square) small_rect(wave, d, a, b);
  a = __builtin_amdgcn_readfirstlane(a);
  b = __builtin_amdgcn_readfirstlane(b);
  const int i = kBandR * a + lane;  // my row (square waves)
  const int j0 = kBandC * b;        // my first column
  const bool row_ok = square && i < d;
  const int q = wave - nrect;                  // diagonal wave index
  const int i0 = kDiagRows * q + lane;         // my two diagonal rows
  const int i1 = i0 + 64;

  v16d s0, s1, s2, s3;
  {
    // unconditional loads from clamped addresses, then a select: no
    // per-element branches
    // entry (i, j) is read from the lower triangle, B[max(i,j)][min(i,j)], so
    // S is bitwise symmetric from the start and stays so (the update
    // fma(-l_i, l_j, s) is symmetric in i and j)
    const int ic = row_ok ? i : 0;
#define LEV_LOAD16(V, OFF)                                                  \
  _Pragma("unroll") for (int e = 0; e < 16; ++e) {                          \
    const int j = j0 + (OFF) + e;                                           \
    const int jc = j < d ? j : 0;                                           \
    const int hi = ic > jc ? ic : jc, lo = ic > jc ? jc : ic;               \
    const double x = B[(int64_t)hi * d + lo];                               \
    V[e] = (row_ok && j < d) ? x : 0.0;                                     \
  }                                                                         \
  __builtin_amdgcn_sched_barrier(0);
    LEV_LOAD16(s0, 0) LEV_LOAD16(s1, 16) LEV_LOAD16(s2, 32) LEV_LOAD16(s3, 48)
#undef LEV_LOAD16
  }
  for (int t = threadIdx.x; t < kLvec; t += blockDim.x) lvec[t] = 0.0;

  // diagonal waves: d_i in registers; leave the wave's candidate
  double dg0 = -INFINITY, dg1 = -INFINITY;
  auto publish_candidate = [&]() {
    const double m = wave_max_f64(fmax(dg0, dg1));
    const unsigned long long h0 = __ballot(dg0 == m && dg0 != -INFINITY);
    const unsigned long long h1 = __ballot(dg1 == m && dg1 != -INFINITY);
    if (lane == 0) {
      Cand cd;
      cd.v = m;
      cd.idx = h0 ? kDiagRows * q + __builtin_ctzll(h0)
                  : (h1 ? kDiagRows * q + 64 + __builtin_ctzll(h1) : 0x7fffffff);
      cand[q] = cd;
    }
  };
  if (!square) {
    if (i0 < d) dg0 = B[(int64_t)i0 * d + i0];
    if (i1 < d) dg1 = B[(int64_t)i1 * d + i1];
    publish_candidate();
  }
  __syncthreads();

  double r00 = 0.0;
  int J = 0;
  for (; J < d; ++J) {
    // the best candidate (larger value, ties to the lower index): all reads
    // issued together
    Cand cs[kSmallD / kDiagRows];
#pragma unroll
    for (int t = 0; t < kSmallD / kDiagRows; ++t) cs[t] = cand[t < ndiag ? t : 0];
    Cand best = cs[0];
#pragma unroll
    for (int t = 1; t < kSmallD / kDiagRows; ++t)
      if (t < ndiag && (cs[t].v > best.v || (cs[t].v == best.v && cs[t].idx < best.idx))) best = cs[t];
    // uniform by construction: kept in scalar registers
    const double pv = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(best.v)),
                                       __builtin_amdgcn_readfirstlane(__double2loint(best.v)));
    const int p = __builtin_amdgcn_readfirstlane(best.idx);
    // 1/sqrt(pv): hardware estimate + two Newton steps (~1 ulp); sqrt = pv/sqrt
    double y = __builtin_amdgcn_rsq(pv);
    y = y * fma(-0.5 * pv * y, y, 1.5);
    y = y * fma(-0.5 * pv * y, y, 1.5);
    y = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(y)),
                         __builtin_amdgcn_readfirstlane(__double2loint(y)));
    const double inv = pv > 0.0 ? y : 0.0;
    const double rpp = pv > 0.0 ? pv * y : 0.0;
    if (J == 0) r00 = rpp;
    if (!(pv > 0.0) || !(rpp > zeta * r00)) break;  // uniform
    if (square) {
      // row p: the lane holding row p in each square with b <= b_p writes
      // its 64 entries (columns >= p duplicate the column-p owners' writes
      // below with identical bits, S being symmetric)
      if (a == p / kBandR && lane == (p & (kBandR - 1)) && b <= p / kBandC) {
        double2* dst = reinterpret_cast<double2*>(&lvec[j0]);
#define LEV_PUT16(V, OFF) \
  _Pragma("unroll") for (int e = 0; e < 16; e += 2) dst[((OFF) + e) / 2] = make_double2(V[e] * inv, V[e + 1] * inv);
        LEV_PUT16(s0, 0) LEV_PUT16(s1, 16) LEV_PUT16(s2, 32) LEV_PUT16(s3, 48)
#undef LEV_PUT16
      }
      // column p, rows i >= p; the entry is picked with a uniform-index
      // register extract
      if (b == p / kBandC) {
        const int cp = __builtin_amdgcn_readfirstlane(p - j0);
        const int e = cp & 15, blk = cp >> 4;
        const double v0 = s0[e], v1 = s1[e], v2 = s2[e], v3 = s3[e];
        const double v = blk == 0 ? v0 : (blk == 1 ? v1 : (blk == 2 ? v2 : v3));
        if (row_ok && i >= p) lvec[i] = v * inv;
      }
    }
    lds_barrier();
    if (square) {
      const double li = row_ok ? lvec[i] : 0.0;
      // 32 groups of 2 columns; the LDS reads of group g + 1 are issued
      // before the FMAs of group g, and each FMA result is pinned in place so
      // the compiler neither sinks the FMAs nor hoists every read of the step
      double lj[2][2];
#define LEV_READ2(buf, OFF) \
  _Pragma("unroll") for (int e = 0; e < 2; ++e) lj[buf][e] = lvec[j0 + (OFF) + e];
#define LEV_FMA2(buf, V, E0)                                               \
  _Pragma("unroll") for (int e = 0; e < 2; ++e) {                          \
    double t = fma(-li, lj[buf][e], V[(E0) + e]);                          \
    asm volatile("" : "+v"(t));                                            \
    V[(E0) + e] = t;                                                       \
  }
      LEV_READ2(0, 0)
      LEV_READ2(1, 2) LEV_FMA2(0, s0, 0)
      LEV_READ2(0, 4) LEV_FMA2(1, s0, 2)
      LEV_READ2(1, 6) LEV_FMA2(0, s0, 4)
      LEV_READ2(0, 8) LEV_FMA2(1, s0, 6)
      LEV_READ2(1, 10) LEV_FMA2(0, s0, 8)
      LEV_READ2(0, 12) LEV_FMA2(1, s0, 10)
      LEV_READ2(1, 14) LEV_FMA2(0, s0, 12)
      LEV_READ2(0, 16) LEV_FMA2(1, s0, 14)
      LEV_READ2(1, 18) LEV_FMA2(0, s1, 0)
      LEV_READ2(0, 20) LEV_FMA2(1, s1, 2)
      LEV_READ2(1, 22) LEV_FMA2(0, s1, 4)
      LEV_READ2(0, 24) LEV_FMA2(1, s1, 6)
      LEV_READ2(1, 26) LEV_FMA2(0, s1, 8)
      LEV_READ2(0, 28) LEV_FMA2(1, s1, 10)
      LEV_READ2(1, 30) LEV_FMA2(0, s1, 12)
      LEV_READ2(0, 32) LEV_FMA2(1, s1, 14)
      LEV_READ2(1, 34) LEV_FMA2(0, s2, 0)
      LEV_READ2(0, 36) LEV_FMA2(1, s2, 2)
      LEV_READ2(1, 38) LEV_FMA2(0, s2, 4)
      LEV_READ2(0, 40) LEV_FMA2(1, s2, 6)
      LEV_READ2(1, 42) LEV_FMA2(0, s2, 8)
      LEV_READ2(0, 44) LEV_FMA2(1, s2, 10)
      LEV_READ2(1, 46) LEV_FMA2(0, s2, 12)
      LEV_READ2(0, 48) LEV_FMA2(1, s2, 14)
      LEV_READ2(1, 50) LEV_FMA2(0, s3, 0)
      LEV_READ2(0, 52) LEV_FMA2(1, s3, 2)
      LEV_READ2(1, 54) LEV_FMA2(0, s3, 4)
      LEV_READ2(0, 56) LEV_FMA2(1, s3, 6)
      LEV_READ2(1, 58) LEV_FMA2(0, s3, 8)
      LEV_READ2(0, 60) LEV_FMA2(1, s3, 10)
      LEV_READ2(1, 62) LEV_FMA2(0, s3, 12)
      LEV_FMA2(1, s3, 14)
#undef LEV_READ2
#undef LEV_FMA2
    } else {
      const double l0 = i0 < d ? lvec[i0] : 0.0;
      const double l1 = i1 < d ? lvec[i1] : 0.0;
      dg0 = (i0 == p) ? -INFINITY : fma(-l0, l0, dg0);
      dg1 = (i1 == p) ? -INFINITY : fma(-l1, l1, dg1);
      if (i0 < d) st.Rrows[(int64_t)J * d + i0] = l0;
      if (i1 < d) st.Rrows[(int64_t)J * d + i1] = l1;
      publish_candidate();
    }
    if (threadIdx.x == 0) st.piv[J] = p;
    lds_barrier();
  }
  if (threadIdx.x == 0) {
    *st.r00 = r00;
    st.flags[0] = 1;
    st.flags[1] = J;
    *rank_out = J;
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
  if (d <= kSmallD) {
    const int waves = small_rects((int)d) + small_diag_waves((int)d);
    pivchol_small_kernel<<<1, 64 * waves, 0, s>>>(B, (int)d, zeta, st, rank_out);
    return hipGetLastError();
  }
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
