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

// Max over lanes 0..7 (row shifts within the first 16-lane row), returned
// to every lane (the workgroup's at most 8 wave candidates).
__device__ __forceinline__ double max8_f64(double v) {
  v = dpp_max_step<0x111, 0xF>(v);  // row_shr:1
  v = dpp_max_step<0x112, 0xF>(v);  // row_shr:2
  v = dpp_max_step<0x114, 0xF>(v);  // row_shr:4
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 7);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 7);
  return __hiloint2double(hi, lo);
}

// One panel of NB pivot steps.  Thread t owns the adjacent columns 2t and
// 2t + 1 (at most 8 waves for d <= 1024): every pivot step runs two
// reductions and two barriers whose cost is paid per wave, so half as many
// waves, each with twice the column work, halve that part of the step.  The
// lane's candidate is the larger of its two diagonals (ties to the lower
// column), the wave's the lowest lane holding the wave max, the workgroup's
// the lowest wave holding the overall max: ties go to the lowest column.
// flags[0] = done, flags[1] = pivots computed so far.
constexpr int kPanelCols = 2;
constexpr int kPanelThreads = kMaxD / kPanelCols;
constexpr int kPanelWaves = kPanelThreads / 64;

// FIXED: the pivot order is the identity (step J's only candidate is column J).
template <bool FIXED>
__global__ __launch_bounds__(kPanelThreads) void pivchol_panel_kernel(const double* __restrict__ S, int64_t d,
                                                                      double zeta, int64_t J0,
                                                                      PivCholState st,
                                                                      int64_t* __restrict__ rank_out,
                                                                      const double* __restrict__ ref_r00) {
  __shared__ double bc[NB];
  __shared__ double wv[2][kPanelWaves];
  __shared__ int wi[2][kPanelWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int c0 = kPanelCols * tid;  // columns c0, c0 + 1
  if (J0 > 0 && st.flags[0] != 0) return;

  double dg[2];
  bool alive[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int c = c0 + q;
    dg[q] = (c < d) ? ((J0 == 0) ? S[(int64_t)c * d + c] : st.diag[c]) : -INFINITY;
    alive[q] = (c < d) && (dg[q] != -INFINITY);
  }
  double r00 = ref_r00 != nullptr ? *ref_r00 : ((J0 == 0) ? 0.0 : *st.r00);
  // the cutoff sqrt(pv) > zeta r00 is tested as pv > (zeta r00)^2, so that
  // no square root stands between the pivot and the exchange of its column
  // (if the square overflows, sqrt(pv) cannot exceed zeta r00 either)
  double zr2 = (zeta * r00) * (zeta * r00);

  double rp0[NB], rp1[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) rp0[t] = rp1[t] = 0.0;

  int64_t J = J0;
  bool stop = false;
  bool active = true;  // uniform across the workgroup
  const int di = (int)d;  // d <= kMaxD: 32-bit offsets below
  double* rrow = st.Rrows + J0 * d + c0;  // row J of R at this thread's columns
  // Constant trip count (no break) so the loop unrolls fully and rp0[],
  // rp1[] stay in registers.
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (active && J >= d) active = false;
    if (!active) continue;
    // the lane's candidate (a column no longer alive holds -inf; fixed
    // order: the only candidate of step J is column J); a NaN diagonal
    // never wins
    const double m0 = (!FIXED || c0 == J) ? dg[0] : -INFINITY;
    const double m1 = (!FIXED || c0 + 1 == J) ? dg[1] : -INFINITY;
    const bool second = (m1 > m0) || (m0 != m0);
    const double mv = second ? m1 : m0;
    const int mc = c0 + (second ? 1 : 0);
    const double wmax = wave_max_f64(mv);
    const uint64_t hit = __ballot(mv == wmax);
    const int hl = hit != 0 ? (__ffsll((unsigned long long)hit) - 1) : 0;
    const int hc = __builtin_amdgcn_readlane(mc, hl);
    if (lane == 0) {
      wv[j & 1][wave] = hit != 0 ? wmax : -INFINITY;
      wi[j & 1][wave] = hit != 0 ? hc : 0x7fffffff;
    }
    // (LDS-only barriers: the R rows this kernel stores are read by later
    // launches only, and waiting for their acknowledgement at every pivot
    // step would put a global-store round trip into each step)
    lds_barrier();
    // the workgroup's pivot, found by every wave: lane w takes wave w's
    // candidate; the largest value wins, ties to the lowest wave (whose
    // columns are the lower ones)
    const double cv = lane < nwaves ? wv[j & 1][lane] : -INFINITY;
    const int ci = lane < nwaves ? wi[j & 1][lane] : 0x7fffffff;
    const double bmax = max8_f64(cv);
    const uint64_t bhit = __ballot(lane < 8 && cv == bmax);
    const int bw = bhit != 0 ? (__ffsll((unsigned long long)bhit) - 1) : 0;
    const double pv = bhit != 0 ? bmax : -INFINITY;
    const int p = __builtin_amdgcn_readlane(ci, bw);
    if (j == 0 && J0 == 0 && ref_r00 == nullptr) {
      r00 = pv > 0.0 ? sqrt(pv) : 0.0;
      zr2 = (zeta * r00) * (zeta * r00);
    }
    if (!(pv > 0.0) || !(pv > zr2)) {
      stop = true;
      active = false;
      continue;
    }
    // prefetch the pivot row of the Schur complement (symmetric: = column p)
    double s_pc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) s_pc[q] = (c0 + q < di) ? S[p * di + c0 + q] : 0.0;
    if ((p >> 1) == tid) {
#pragma unroll
      for (int t = 0; t < j; ++t) bc[t] = (p & 1) ? rp1[t] : rp0[t];
    }
    lds_barrier();
    // rjj and 1 / rjj (the reciprocal estimate and two Newton steps: rjj is
    // positive, finite and normal here, so the scaled division's special
    // cases do not arise) while the column's entries are read and summed
    const double rjj = sqrt(pv);
    double inv = __builtin_amdgcn_rcp(rjj);
    inv = fma(inv, fma(-rjj, inv, 1.0), inv);
    inv = fma(inv, fma(-rjj, inv, 1.0), inv);
    double acc0 = s_pc[0], acc1 = s_pc[1];
#pragma unroll
    for (int t = 0; t < j; ++t) {
      const double b = bc[t];
      acc0 = fma(-b, rp0[t], acc0);
      acc1 = fma(-b, rp1[t], acc1);
    }
    // selects, not branches: the pivot column takes rjj and leaves the
    // candidates, live columns take their entry and downdate their diagonal,
    // dead ones (and those past d) take 0
    double val[2] = {acc0 * inv, acc1 * inv};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool piv = c0 + q == p;
      const double nd = fma(-val[q], val[q], dg[q]);
      val[q] = piv ? rjj : (alive[q] ? val[q] : 0.0);
      dg[q] = piv ? -INFINITY : (alive[q] ? nd : dg[q]);
      alive[q] = alive[q] && !piv;
    }
    rp0[j] = val[0];
    rp1[j] = val[1];
    if (c0 + 1 < d && ((d & 1) == 0)) {  // the pair is 16-byte aligned (d even, c0 even)
      *reinterpret_cast<double2*>(rrow) = make_double2(val[0], val[1]);
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (c0 + q < d) rrow[q] = val[q];
    }
    rrow += d;
    if (tid == 0) st.piv[J] = p;
    ++J;
  }

#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (c0 + q < d) st.diag[c0 + q] = dg[q];
  if (tid == 0) {
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
// holds the 8 x 8 block of rows 64a + 8 (l / 8) + 0..7 and columns
// 64b + 8 (l % 8) + 0..7 in 128 registers, so a row and a column of the square
// are both spread over 8 lanes.  One more, the "diagonal" wave, owns the
// Schur diagonal: lane l holds d_i for rows i = l + 64 t (t < 4), updated as
// d_i -= l_i^2.  Eleven waves (at most three per SIMD) leave up to 170
// registers per lane.
//
// Per pivot step (two barriers): the square waves read the pivot p and
// 1/sqrt(S_pp) that the diagonal wave posted; column p of the squares
// (a, b_p) gives l for the bands >= b_p and row p of the squares (b_p, b),
// b < b_p, gives it for the bands below (each entry written once, 8 lanes x
// 8 values per square), l = S[:, p] / sqrt(S_pp) going to LDS; after the
// barrier the square waves apply S -= l l^T to their entries (8 + 8 values of
// l per lane, 64 FMAs) while the diagonal wave, at the same time and first in
// issue, updates d, stores R[J, :] = l and posts the next pivot: the argmax of
// d (DPP wave reduction, ties to the lower index) and its 1/sqrt from the
// hardware estimate plus two Newton steps.  No global memory is read inside
// the loop.
constexpr int kSmallD = 256;
// Bound on the pivot wait.  The wait ends by construction (see the loop);
// if the bound is ever reached the wave sets kErrPivotWait in st.err and
// stops, so the call's results are flagged instead of silently wrong.
constexpr int kSpinLimit = 1 << 22;
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


// The pivot of the next step, posted by the diagonal wave.
struct __align__(16) PivotMsg {
  double inv;  // 1 / sqrt(S_pp)
  int p;
  int ok;  // 0: the factorization stops here
};

__global__ __launch_bounds__(768) void pivchol_small_kernel(const double* __restrict__ B, int d, double zeta,
                                                            PivCholState st, int64_t* __restrict__ rank_out,
                                                            int fixed, const double* __restrict__ ref_r00) {
  // step J uses lvec[J & 1] and msg[J & 1]; `posted` counts the pivots the
  // diagonal wave has posted (msg[J & 1] holds pivot J once posted > J)
  __shared__ __align__(16) double lvec[2][kLvec];
  __shared__ PivotMsg msg[2];
  __shared__ int posted;

  const int lane = threadIdx.x & 63;
  // wave-uniform values kept scalar (the compiler cannot infer it)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nrect = small_rects(d);
  const bool square = wave < nrect;  // uniform; the last wave is the diagonal one
  int a = 0, b = 0;
  if (square) small_rect(wave, d, a, b);
  a = __builtin_amdgcn_readfirstlane(a);
  b = __builtin_amdgcn_readfirstlane(b);
  // square waves: lane l holds the 8 x 8 block rows ri0 .. ri0 + 7, columns
  // cj0 .. cj0 + 7 of the square (a, b); entry (r, c) is element (r % 2) * 8 + c
  // of vector r / 2
  const int gr = lane >> 3, gc = lane & 7;
  const int ri0 = kBandR * a + 8 * gr;
  const int cj0 = kBandC * b + 8 * gc;

  v16d s0, s1, s2, s3;
  {
    // unconditional loads from clamped addresses, then a select: no
    // per-element branches
    // entry (i, j) is read from the lower triangle, B[max(i,j)][min(i,j)], so
    // S is bitwise symmetric from the start and stays so (the update
    // fma(-l_i, l_j, s) is symmetric in i and j)
#define LEV_LOAD16(V, R0)                                                   \
  _Pragma("unroll") for (int e = 0; e < 16; ++e) {                          \
    const int i = ri0 + (R0) + e / 8, j = cj0 + e % 8;                      \
    const bool ok = square && i < d && j < d;                               \
    const int ic = ok ? i : 0, jc = ok ? j : 0;                             \
    const int hi = ic > jc ? ic : jc, lo = ic > jc ? jc : ic;               \
    const double x = B[(int64_t)hi * d + lo];                               \
    V[e] = ok ? x : 0.0;                                                    \
  }                                                                         \
  __builtin_amdgcn_sched_barrier(0);
    LEV_LOAD16(s0, 0) LEV_LOAD16(s1, 2) LEV_LOAD16(s2, 4) LEV_LOAD16(s3, 6)
#undef LEV_LOAD16
  }
  for (int t = threadIdx.x; t < 2 * kLvec; t += blockDim.x) lvec[t / kLvec][t % kLvec] = 0.0;

  if (square) {
    __syncthreads();  // the first pivot is posted
    for (int J = 0; J < d; ++J) {
      // pivot J: posted by the diagonal wave once every wave has passed the
      // barrier of step J - 1, which this wave has, so the wait ends.
      // The counter is read with acquire semantics and the diagonal wave
      // stores it with release semantics after the message, so a counter
      // that shows pivot J makes message J visible to the loads behind it.
      uint64_t m0 = 0, m1 = 0;
      bool timed_out = false;
      for (int spin = 0;; ++spin) {
        const int seen = __hip_atomic_load(&posted, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        uint64_t* mp = reinterpret_cast<uint64_t*>(&msg[J & 1]);
        m0 = __hip_atomic_load(mp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        m1 = __hip_atomic_load(mp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (seen > J) break;
        if (spin >= kSpinLimit) {
          timed_out = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (timed_out) {
        if (lane == 0 && st.err != nullptr)
          __hip_atomic_fetch_or(st.err, kErrPivotWait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;  // this wave leaves the factorization; the call is flagged
      }
      const int p = __builtin_amdgcn_readfirstlane((int)(uint32_t)m1);
      const int ok = __builtin_amdgcn_readfirstlane((int)(uint32_t)(m1 >> 32));
      const double inv = __hiloint2double(__builtin_amdgcn_readfirstlane((int)(uint32_t)(m0 >> 32)),
                                          __builtin_amdgcn_readfirstlane((int)(uint32_t)m0));
      if (!ok) break;
      double* lv = lvec[J & 1];
      const int bp = p / kBandC;
      const int pl = p - kBandC * bp;  // p's position inside its band
      if (b == bp) {
        // column p of the squares (a, b_p), a >= b_p: rows of bands >= b_p;
        // the 8 lanes of column group pl / 8 each hold 8 rows of it (entry
        // (r, c) of the lane's block is element (r % 2) * 8 + c of vector
        // r / 2), picked by a uniform switch on c
        if (gc == (pl >> 3)) {
          double v[8];
          switch (__builtin_amdgcn_readfirstlane(pl & 7)) {
#define LEV_COL(C)                                                                                  \
  case C:                                                                                           \
    v[0] = s0[C], v[1] = s0[8 + C], v[2] = s1[C], v[3] = s1[8 + C];                                 \
    v[4] = s2[C], v[5] = s2[8 + C], v[6] = s3[C], v[7] = s3[8 + C];                                 \
    break;
            LEV_COL(0) LEV_COL(1) LEV_COL(2) LEV_COL(3) LEV_COL(4) LEV_COL(5) LEV_COL(6) default: LEV_COL(7)
#undef LEV_COL
          }
          double2* dst = reinterpret_cast<double2*>(&lv[ri0]);
#pragma unroll
          for (int q = 0; q < 4; ++q) dst[q] = make_double2(v[2 * q] * inv, v[2 * q + 1] * inv);
        }
      } else if (a == bp) {
        // row p of the squares (b_p, b), b < b_p: columns of bands < b_p,
        // by symmetry the entries of column p there; row r = pl % 8 of the
        // lane's block is elements (r % 2) * 8 .. + 7 of vector r / 2
        if (gr == (pl >> 3)) {
          double w[8];
          switch (__builtin_amdgcn_readfirstlane(pl & 7)) {
#define LEV_ROW(R, V)                                                                               \
  case R:                                                                                           \
    _Pragma("unroll") for (int c = 0; c < 8; ++c) w[c] = V[((R) & 1) * 8 + c];                      \
    break;
            LEV_ROW(0, s0) LEV_ROW(1, s0) LEV_ROW(2, s1) LEV_ROW(3, s1) LEV_ROW(4, s2) LEV_ROW(5, s2)
            LEV_ROW(6, s3) default: LEV_ROW(7, s3)
#undef LEV_ROW
          }
          double2* dst = reinterpret_cast<double2*>(&lv[cj0]);
#pragma unroll
          for (int c = 0; c < 8; c += 2) dst[c / 2] = make_double2(w[c] * inv, w[c + 1] * inv);
        }
      }
      lds_barrier();
      // S -= l l^T on the lane's 8 x 8 block: 8 column values and 8 row
      // values of l, 64 FMAs (each result pinned so that the compiler keeps
      // the FMAs where they are)
      double lc[8], lr[4];
      {
        const double2* src = reinterpret_cast<const double2*>(&lv[cj0]);
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
          const double2 t = src[c / 2];
          lc[c] = t.x;
          lc[c + 1] = t.y;
        }
      }
      const double2* srr = reinterpret_cast<const double2*>(&lv[ri0]);
#define LEV_ROWS4(R0)                                                      \
  {                                                                        \
    const double2 t0 = srr[(R0) / 2], t1 = srr[(R0) / 2 + 1];              \
    lr[0] = t0.x;                                                          \
    lr[1] = t0.y;                                                          \
    lr[2] = t1.x;                                                          \
    lr[3] = t1.y;                                                          \
  }
#define LEV_UPD16(V, R)                                                    \
  _Pragma("unroll") for (int e = 0; e < 16; ++e) {                         \
    double t = fma(-lr[(R) + e / 8], lc[e % 8], V[e]);                     \
    asm volatile("" : "+v"(t));                                            \
    V[e] = t;                                                              \
  }
      LEV_ROWS4(0) LEV_UPD16(s0, 0) LEV_UPD16(s1, 2)
      LEV_ROWS4(4) LEV_UPD16(s2, 0) LEV_UPD16(s3, 2)
#undef LEV_ROWS4
#undef LEV_UPD16
      if (threadIdx.x == 0) st.piv[J] = p;
    }
  } else {
    // the diagonal wave: d_i for rows lane + 64 t; the serial part of each
    // pivot, so first in issue
    __builtin_amdgcn_s_setprio(3);
    double dg[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = lane + 64 * t;
      dg[t] = i < d ? B[(int64_t)i * d + i] : -INFINITY;
    }
    double r00 = ref_r00 != nullptr ? *ref_r00 : 0.0;
    int cur_p = 0;
    // posts the pivot of step J: the largest d_i, ties to the lower index
    // (fixed order: d_J), with 1/sqrt(d_p) (hardware estimate + two Newton
    // steps, ~1 ulp); returns whether the factorization continues
    auto post = [&](int J) -> bool {
      double cand[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) cand[t] = (!fixed || lane + 64 * t == J) ? dg[t] : -INFINITY;
      const double m = wave_max_f64(fmax(fmax(cand[0], cand[1]), fmax(cand[2], cand[3])));
      int p = 0x7fffffff;
#pragma unroll
      for (int t = 3; t >= 0; --t) {
        const unsigned long long h = __ballot(cand[t] == m && cand[t] != -INFINITY);
        if (h) p = 64 * t + __builtin_ctzll(h);
      }
      p = __builtin_amdgcn_readfirstlane(p);
      const double pv = m;
      double y = __builtin_amdgcn_rsq(pv);
      y = y * fma(-0.5 * pv * y, y, 1.5);
      y = y * fma(-0.5 * pv * y, y, 1.5);
      const double inv = pv > 0.0 ? y : 0.0;
      const double rpp = pv > 0.0 ? pv * y : 0.0;
      if (J == 0 && ref_r00 == nullptr) r00 = rpp;
      const bool ok = pv > 0.0 && rpp > zeta * r00;
      if (lane == 0) {
        PivotMsg pm;
        pm.inv = inv;
        pm.p = p;
        pm.ok = ok ? 1 : 0;
        msg[J & 1] = pm;
        __hip_atomic_store(&posted, J + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      cur_p = p;
      return ok;
    };
    bool ok = post(0);
    __syncthreads();
    int J = 0;
    for (; J < d && ok; ++J) {
      const int p = cur_p;
      lds_barrier();
      // all four reads in flight at once (lvec holds kLvec >= 4 * 64 entries,
      // zero past d), the next pivot posted before the stores of R's row
      const double* lv = lvec[J & 1];
      double l[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) l[t] = lv[lane + 64 * t];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = lane + 64 * t;
        dg[t] = (i == p || i >= d) ? -INFINITY : fma(-l[t], l[t], dg[t]);
      }
      ok = post(J + 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = lane + 64 * t;
        if (i < d) st.Rrows[(int64_t)J * d + i] = l[t];
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (lane == 0) {
      *st.r00 = r00;
      st.flags[0] = 1;
      st.flags[1] = J;
      *rank_out = J;
    }
  }
}

// perm: pivots, then the unselected columns ascending.  R_out: pivoted,
// upper triangular, rows >= r zero.  One launch: every workgroup rebuilds
// the permutation in LDS (a ballot count of the unselected columns per wave,
// then a sum over the waves before it), workgroup 0 writes it out, and each
// workgroup gathers kFinalRows rows of R.
constexpr int kFinalRows = 4;

__global__ __launch_bounds__(kMaxD) void pivchol_finalize_kernel(int64_t d, PivCholState st,
                                                                 const int64_t* __restrict__ rank,
                                                                 int32_t* __restrict__ perm_out,
                                                                 double* __restrict__ R_out) {
  __shared__ int chosen[kMaxD];
  __shared__ int wave_cnt[kMaxD / 64];
  __shared__ int perm_s[kMaxD];
  const int c = threadIdx.x;
  const int lane = c & 63, w = c >> 6;
  const int64_t r = *rank;  // 0 <= r <= d
  chosen[c] = 0;
  __syncthreads();
  if (c < r) chosen[st.piv[c]] = 1;
  __syncthreads();
  const bool free_c = c < d && chosen[c] == 0;
  const unsigned long long bal = __ballot(free_c);
  if (lane == 0) wave_cnt[w] = __popcll(bal);
  __syncthreads();
  int before = __popcll(bal & ((1ull << lane) - 1ull));
  for (int q = 0; q < w; ++q) before += wave_cnt[q];
  if (c < r) perm_s[c] = st.piv[c];
  if (free_c) perm_s[r + before] = c;
  __syncthreads();
  if (blockIdx.x == 0 && c < d) perm_out[c] = perm_s[c];
  const int64_t j0 = (int64_t)blockIdx.x * kFinalRows;
  const int64_t j1 = j0 + kFinalRows < d ? j0 + kFinalRows : d;
  for (int64_t j = j0; j < j1; ++j)
    for (int64_t t = c; t < d; t += kMaxD) {
      double v = 0.0;
      if (j < r && t >= j) v = st.Rrows[j * d + perm_s[t]];
      R_out[j * d + t] = v;
    }
}

// Rank-NB update after a panel: S <- S - R_p^T R_p, R_p the panel's NB rows
// of R (NB x d, row-major).  One K step of NB, so a tiled GEMM would spend
// its time on the LDS staging and barrier around a single step; here there
// is no LDS: each wave owns a 32 x 32 block of S (2 x 2 blocks of the 16x16x4
// FP64 MFMA), loads the R values of its operands straight into registers
// (16 lanes read 128 contiguous bytes of one row of R_p) together with its
// block of S, runs the NB / 4 MFMA steps and writes S - (R_p^T R_p) back,
// the same arithmetic as the GEMM form: the product summed from zero in
// k order, then one subtraction.  Skipped once the factorisation is done.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kSchurTile = 64;  // rows and columns of S per workgroup (4 waves)

__global__ __launch_bounds__(256) void schur_update_kernel(double* __restrict__ S, int64_t d,
                                                           const double* __restrict__ Rp,
                                                           const int32_t* __restrict__ done) {
  if (*done != 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.y * kSchurTile + (wave >> 1) * 32;
  const int64_t c0 = (int64_t)blockIdx.x * kSchurTile + (wave & 1) * 32;
  // operands of step s (contraction index k = 4 s + g): lane l supplies
  // A[l % 16][l / 16] = R_p[k][r0 + 16 bi + l % 16] and B[l / 16][l % 16] =
  // R_p[k][c0 + 16 bj + l % 16]; indices past d read zero
  double av[NB / 4][2], bv[NB / 4][2];
#pragma unroll
  for (int st = 0; st < NB / 4; ++st)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double* row = Rp + (int64_t)(4 * st + g) * d;
      const int64_t ri = r0 + 16 * h + i, cj = c0 + 16 * h + i;
      av[st][h] = ri < d ? row[ri] : 0.0;
      bv[st][h] = cj < d ? row[cj] : 0.0;
    }
  // S block: accumulator element v of lane l is row g + 4 v, column i
  double sv[2][2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + 16 * bi + g + 4 * v, c = c0 + 16 * bj + i;
        sv[bi][bj][v] = (r < d && c < d) ? S[r * d + c] : 0.0;
      }
  v4d acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < NB / 4; ++st)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st][bi], bv[st][bj], acc[bi][bj], 0, 0, 0);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + 16 * bi + g + 4 * v, c = c0 + 16 * bj + i;
        if (r < d && c < d) S[r * d + c] = sv[bi][bj][v] - acc[bi][bj][v];
      }
}

}  // namespace

hipError_t launch_pivchol(double* B, int64_t d, double zeta, const PivCholState& st, int64_t* rank_out,
                          double* gemm_partial, hipStream_t s, int fixed, const double* ref_r00) {
  (void)gemm_partial;
  if (d <= 0 || d > kMaxD) return hipErrorInvalidValue;
  if (d <= kSmallD) {
    const int waves = small_rects((int)d) + 1;
    pivchol_small_kernel<<<1, 64 * waves, 0, s>>>(B, (int)d, zeta, st, rank_out, fixed, ref_r00);
    return hipGetLastError();
  }
  const int threads = (int)(((d + 64 * kPanelCols - 1) / (64 * kPanelCols)) * 64);
  for (int64_t J0 = 0; J0 < d; J0 += NB) {
    if (fixed)
      pivchol_panel_kernel<true><<<1, threads, 0, s>>>(B, d, zeta, J0, st, rank_out, ref_r00);
    else
      pivchol_panel_kernel<false><<<1, threads, 0, s>>>(B, d, zeta, J0, st, rank_out, ref_r00);
    if (J0 + NB < d) {
      // S <- S - R_panel^T R_panel over the panel's NB rows (skipped once done)
      const double* Rp = st.Rrows + J0 * d;
      const unsigned tiles = (unsigned)((d + kSchurTile - 1) / kSchurTile);
      schur_update_kernel<<<dim3(tiles, tiles), 256, 0, s>>>(B, d, Rp, st.flags);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_pivchol_finalize(int64_t d, const PivCholState& st, const int64_t* rank,
                                   int32_t* perm_out, double* R_out, hipStream_t s) {
  if (d <= 0 || d > kMaxD) return hipErrorInvalidValue;
  pivchol_finalize_kernel<<<(unsigned)((d + kFinalRows - 1) / kFinalRows), kMaxD, 0, s>>>(d, st, rank, perm_out,
                                                                                          R_out);
  return hipGetLastError();
}

}  // namespace lev
