// Algorithm 8, step 4, on the selected columns: X = R~^{-1} Pi_2, here
// Z = R11^{-1} G_k[0:r, :] by back substitution in FP64 (R11 is the leading
// r x r block of the pivoted factor; r is read on the device), then Z is
// scattered to the original column ids (Z_full[perm[j], :] = Z[j, :], zero
// rows off K) and converted to the operand layout of pass 2.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lev_internal.h"

namespace lev {
namespace {

// A diagonal block of at most 256 pivot positions (all of R11 when
// r <= 256): one workgroup of 16 waves solves R11 Z = G for a group of 64
// right-hand sides (columns c0 .. c0 + 63) by blocked back substitution with
// inverted diagonal blocks, all products on 16 x 16 x 4 FP64 MFMAs.  Wave w
// owns row block w (rows 16 w .. 16 w + 15):
//   T_w = R_ww^{-1}                    (one column per lane, 16 lanes)
//   Z_w = T_w G_w - sum_{b > w} (T_w R_wb) Z_b
// The wave starts from Y = T_w G_w and, for b = nblk - 1 down to w + 1,
// forms M_b = T_w R_wb from R (loaded one block ahead), waits for the owner
// of block b to publish Z_b, and subtracts M_b Z_b; then it publishes Z_w.
// Every Z_b keeps its own LDS slot and a ready flag, so the waves run at
// their own pace and the serial chain from one owner to the next is a single
// set of MFMAs (M_b is formed while Z_b is pending).  Operand layouts
// (lane l, kk = l / 16, i = l % 16): the accumulator holds element (l / 16 +
// 4 v, l % 16) of each 16 x 16 column block; its element v is exactly the B
// operand of k-step v, so Y and M_b take T_w as A and the accumulator (or R's
// block loaded in that order) as B.  The update's k-step q takes column
// 4 kk + q: A = -M_b[i][4 kk + q] (the accumulator of M_b re-read through
// LDS), B = Z_b[4 kk + q][16 cb + i], which the owner published at lane
// 16 q + i, element kk.  Once every block is out, the workgroup writes Z and
// (form_z) the pass-2 operand from LDS with 16-byte stores.
constexpr int kTrsmR = 256;
constexpr int kDiagDoubles = (kTrsmR / 16) * 16 * 16;
constexpr int kZallDoubles = (kTrsmR / 16) * 4 * 4 * 64;  // every Z_b, KB <= 4
constexpr int kSolveLdsDoubles = kZallDoubles;            // 128 KB; the diagonal blocks first
// Bound on a flag wait.  The waits end by construction (a block only waits
// on later ones, whose owners never wait on it); if the bound is ever
// reached the wave sets kErrSolveWait in the error word, stops updating and
// publishes what it has, so no other wave waits on it and the call is
// flagged instead of silently wrong.
constexpr int kSpinLimit = 1 << 22;
typedef double v4d __attribute__((ext_vector_type(4)));

// Pass-2 operand layouts (see rownorm.hip).  For chunk t of the contraction
// (CW columns), column tile cb (16 output columns), lane l and element e:
//   value = Z_full[t*CW + EL*(l/16) + e][16*cb + (l%16)]
// stored at ((t*CB + cb)*64 + l)*EL + e, CB = ceil(k/16).
//   FP64: EL = 2, CW = 8.   FP32: EL = 4, CW = 16.   BF16 forms: EL = 8, CW = 32.
// BF16 forms store NP parts one after the other, split in FP32: x = float(v),
// part 0 = RNE(x), part p = RNE(x - parts 0..p-1) (each difference is exact in
// FP32; NP = 1 BF16, 2 BF16 hi/lo, 3 BF16x3: the three parts hold x to ~2^-27,
// below the 2^-24 of the conversion to FP32).
// The CSR forms (variants 5, 6: FP32, FP64) are Z_full row-major with rows
// padded to 64 columns.
template <int VARIANT>
struct PackForm {
  static constexpr bool kRowMajor = VARIANT >= 5;
  static constexpr int EL = VARIANT == 0 ? 2 : (VARIANT == 1 ? 4 : 8);
  static constexpr int CW = 4 * EL;
  static constexpr int NP = VARIANT == 3 ? 2 : (VARIANT == 4 ? 3 : 1);
  using OUT = typename std::conditional<
      VARIANT == 0 || VARIANT == 6, double,
      typename std::conditional<VARIANT == 1 || VARIANT == 5, float, __hip_bfloat16>::type>::type;
  // elements per 16-byte store
  static constexpr int kVec = 16 / sizeof(OUT);
};

// LDS slot of Z[j][c] (pivot position j < r, column c < 16 KB) as published.
template <int KB>
__device__ __forceinline__ int zall_index(int j, int c) {
  const int b = j >> 4, i = j & 15;
  return b * (4 * KB * 64) + ((i >> 2) * KB + (c >> 4)) * 64 + 16 * (i & 3) + (c & 15);
}

// Solves for the workgroup's 64 columns; ends with every Z_b in zall (lds)
// and a workgroup barrier.  lds holds kSolveLdsDoubles doubles, ready 16
// flags.  KB = ceil(min(k - c0, 64) / 16) column blocks of 16 (a template
// parameter: a run-time bound on the accumulator blocks makes the compiler
// copy them).
template <int KB>
__device__ __forceinline__ void blocked_solve(double* lds, int32_t* ready, int d, int k, int c0,
                                              const double* __restrict__ R, int r,
                                              const double* __restrict__ G, int32_t* err) {
  double* rdg = lds;   // prologue: [16][256], diagonal block b, then T_b; then the wave's scratch
  double* zall = lds;  // [16][4][KB][64]: Z_b in the B-operand order
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nblk = (r + 15) / 16;
  if (threadIdx.x < 16) ready[threadIdx.x] = 0;
  // addresses as a uniform row pointer plus a 32-bit lane offset (every
  // operand here is below 2^19 elements)
  // the wave's rows of G, issued first (their latency overlaps the staging;
  // with 4 column blocks they would not fit the registers of the inversion
  // below and are loaded after it)
  v4d acc[KB];
  auto load_g = [&]() {
#pragma unroll
    for (int cb = 0; cb < KB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * w + (lane >> 4) + 4 * v, col = c0 + 16 * cb + (lane & 15);
        acc[cb][v] = (row < r && col < k) ? G[(unsigned)(row * k + col)] : 0.0;
      }
  };
  if constexpr (KB <= 3) load_g();
  // R's blocks above the diagonal, touched once here so that the loads of
  // the loop (one block ahead) hit the L2 cache of this die
  if (nblk > 1) {
    // both ends of each 16-column row segment (one or two cache lines)
    const int rows = 16 * (nblk - 1), segs = 2 * (nblk - 1);
    double sink = 0.0;
#pragma unroll 8
    for (int i = threadIdx.x; i < rows * segs; i += 1024) {
      const int t = i / segs, sg = i % segs;
      sink += R[(unsigned)(t * d + 16 * (sg / 2 + 1) + 15 * (sg & 1))];
    }
    asm volatile("" ::"v"(sink));
  }
  // diagonal blocks: rdg[b][s][e] = R[16 b + e][16 b + s] (e < s), 1 / R_jj at
  // e = s; zero past the rank
  for (int idx = threadIdx.x; idx < nblk * 256; idx += 1024) {
    const int b = idx >> 8, s = (idx >> 4) & 15, e = idx & 15;
    const int i = 16 * b + e, j = 16 * b + s;
    double v = 0.0;
    if (e <= s && j < r) {
      const double x = R[(unsigned)(i * d + j)];
      v = e == s ? 1.0 / x : x;
    }
    rdg[idx] = v;
  }
  // LDS-only barrier (no wait for the global loads in flight)
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");

  if (w < nblk) {
    double* rb = rdg + w * 256;
    // T_w: lane j < 16 solves for column j, right-looking, two steps per
    // batch (both columns of R read first, one wait); only 16 lanes run it,
    // since the R values are the same for every lane.  Rows and columns past
    // the rank come out zero.  Written over the wave's own diagonal block
    // (read completely first, LDS order within a wave), then read back as the
    // A operand of k-step q: ta[q] = T_w[l % 16][4 q + l / 16].
    if (lane < 16) {
      const int j = lane;
      double g[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) g[s] = s == j ? 1.0 : 0.0;
#pragma unroll
      for (int s = 15; s >= 1; s -= 2) {
        double c0v[16], c1v[16];
#pragma unroll
        for (int e = 0; e <= s; ++e) c0v[e] = rb[s * 16 + e];
#pragma unroll
        for (int e = 0; e < s; ++e) c1v[e] = rb[(s - 1) * 16 + e];
        __builtin_amdgcn_sched_barrier(0);
        g[s] *= c0v[s];
#pragma unroll
        for (int e = 0; e < s; ++e) g[e] = fma(-c0v[e], g[s], g[e]);
        g[s - 1] *= c1v[s - 1];
#pragma unroll
        for (int e = 0; e < s - 1; ++e) g[e] = fma(-c1v[e], g[s - 1], g[e]);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) rb[j * 16 + i] = g[i];  // T[i][j]
    }
    if constexpr (KB > 3) load_g();
    double ta[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ta[q] = rb[(4 * q + (lane >> 4)) * 16 + (lane & 15)];
    // Y = T_w G_w
    v4d z[KB];
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      z[cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) z[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[q], acc[cb][q], z[cb], 0, 0, 0);
    }
    // R_wb in the B-operand order of k-step q: R[16 w + 4 q + l / 16][16 b + l % 16]
    // (columns past the rank zeroed: they meet zero rows of Z_b anyway)
    auto load_rb = [&](double (&rv)[4], int b) {
      const int col = 16 * b + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * w + 4 * q + (lane >> 4);
        rv[q] = col < r ? R[(unsigned)(row * d + col)] : 0.0;
      }
    };
    double rn[4];
    if (nblk - 1 > w) load_rb(rn, nblk - 1);
    for (int b = nblk - 1; b > w; --b) {
      double rv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) rv[q] = rn[q];
      if (b - 1 > w) load_rb(rn, b - 1);
      // M_b = T_w R_wb, then through the scratch into the update's A order
      v4d m = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) m = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[q], rv[q], m, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) rb[((lane >> 4) + 4 * v) * 16 + (lane & 15)] = m[v];
      double ma[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) ma[q] = -rb[(lane & 15) * 16 + 4 * (lane >> 4) + q];
      // the next owner's last wait is the serial chain
      if (b == w + 1) __builtin_amdgcn_s_setprio(3);
      bool timed_out = false;
      for (int spin = 0; __hip_atomic_load(ready + b, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0;
           ++spin) {
        if (spin >= kSpinLimit) {
          timed_out = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (timed_out) {
        if (lane == 0 && err != nullptr)
          __hip_atomic_fetch_or(err, kErrSolveWait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      const double* zb = zall + b * (4 * KB * 64) + (lane >> 4) * KB * 64 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb)
          z[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[q], zb[cb * 64 + 16 * q], z[cb], 0, 0, 0);
    }
    // publish Z_w in the B-operand order of the updates
    double* zw = zall + w * (4 * KB * 64);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int cb = 0; cb < KB; ++cb) zw[(v * KB + cb) * 64 + lane] = z[cb][v];
    __hip_atomic_store(ready + w, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_s_setprio(0);
  }
  // (The slots of blocks above w never overlap the diagonal block of w, and
  // a slot below w is written only after its owner waited for block w, so
  // the staged blocks and scratch are never overwritten while in use.)
  __syncthreads();
}

// Z (pivot positions 0 .. d - 1, columns c0 .. c0 + 63, c < k) from zall to
// Z64 (row stride k); rows r .. d - 1 zero.  Wave w writes rows w, w + 16, ...
// with one column per lane.
template <int KB>
__device__ __forceinline__ void store_z64(const double* zall, int d, int k, int c0, int r,
                                          double* __restrict__ Z64) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (c0 + lane >= k) return;
  const unsigned c = (unsigned)(c0 + lane);
#pragma unroll 4
  for (int j = w; j < d; j += 16) (Z64 + (int64_t)j * k)[c] = j < r ? zall[zall_index<KB>(j, lane)] : 0.0;
}

// The pass-2 operand of Z_full (Z_full[row] = Z[inv[row]], zero off K), one
// 16-byte piece per thread and part.
template <int VARIANT, int KB>
__device__ __forceinline__ void store_operand(const double* zall, const int32_t* inv, int d, int total,
                                              void* __restrict__ Zpack) {
  using F = PackForm<VARIANT>;
  using OUT = typename F::OUT;
  constexpr int V = F::kVec;
  OUT* out = static_cast<OUT*>(Zpack);
  for (int p0 = threadIdx.x * V; p0 < total; p0 += 1024 * V) {
    double x[V];
    if constexpr (F::kRowMajor) {
      const int row = p0 >> 6, col = p0 & 63;  // V consecutive columns
      const int j = inv[row];
#pragma unroll
      for (int e = 0; e < V; ++e) x[e] = (j >= 0 && col + e < 16 * KB) ? zall[zall_index<KB>(j, col + e)] : 0.0;
    } else {
      // V == EL: the EL consecutive elements e of one (t, cb, l)
      const int l = (p0 / F::EL) % 64, q = p0 / (F::EL * 64);
      const int cb = q % KB, t = q / KB;  // KB column tiles (k <= 64)
      const int row0 = t * F::CW + F::EL * (l / 16), col = 16 * cb + (l % 16);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int row = row0 + e;
        const int j = row < d ? inv[row] : -1;
        x[e] = j >= 0 ? zall[zall_index<KB>(j, col)] : 0.0;
      }
    }
    if constexpr (sizeof(OUT) == 2) {
      float xf[V];
#pragma unroll
      for (int e = 0; e < V; ++e) xf[e] = (float)x[e];
#pragma unroll
      for (int p = 0; p < F::NP; ++p) {
        __hip_bfloat16 h[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          h[e] = __float2bfloat16(xf[e]);
          xf[e] -= __bfloat162float(h[e]);
        }
        *reinterpret_cast<uint4*>(out + p * total + p0) = *reinterpret_cast<const uint4*>(h);
      }
    } else {
      OUT o[V];
#pragma unroll
      for (int e = 0; e < V; ++e) o[e] = (OUT)x[e];
      *reinterpret_cast<uint4*>(out + p0) = *reinterpret_cast<const uint4*>(o);
    }
  }
}

// The diagonal block of pivot positions j0 .. j0 + 255 (fewer at the end of
// d) of R11 Z = G, for k <= 64 columns per workgroup (grid.y groups of 64;
// every group has 4 column blocks, the last one possibly partly past k).  G
// holds the right-hand side of these rows with the contributions of the
// blocks below already subtracted; the rank is read here, so a block wholly
// past it writes zero rows of Z.
__global__ __launch_bounds__(1024) void trsm_blocked_kernel(int64_t d, int64_t k, int64_t j0,
                                                            const double* __restrict__ R,
                                                            const int64_t* __restrict__ rank,
                                                            const double* __restrict__ G,
                                                            double* __restrict__ Z64, int32_t* err) {
  __shared__ double lds[kSolveLdsDoubles];
  __shared__ int32_t ready[16];
  const int c0 = 64 * (int)blockIdx.y;
  const int rows = (int)std::min<int64_t>(kTrsmR, d - j0);
  const int r = (int)std::min<int64_t>(rows, std::max<int64_t>(0, *rank - j0));
  blocked_solve<4>(lds, ready, (int)d, (int)k, c0, R + j0 * d + j0, r, G + j0 * k, err);
  store_z64<4>(lds, rows, (int)k, c0, r, Z64 + j0 * k);
}

// Value of packed element idx (see the layouts above); inv maps a column id
// to its pivot position (-1 off K), zsrc is r x k by pivot position (row
// stride zstride).  (32-bit index arithmetic: the operand has at most 2^18
// elements.)
template <typename OUT, int EL, int NP>
__device__ __forceinline__ void pack_element(int idx, int total, int d, int k, int cbn, const int32_t* inv,
                                             const double* zsrc, int zstride, OUT* out) {
  constexpr int CW = 4 * EL;
  const int e = idx % EL;
  const int l = (idx / EL) % 64;
  const int q = idx / (EL * 64);
  const int cb = q % cbn;
  const int t = q / cbn;
  const int row = t * CW + EL * (l / 16) + e;  // original column id of A
  const int col = 16 * cb + (l % 16);
  double v = 0.0;
  if (row < d && col < k) {
    const int32_t j = inv[row];  // pivot position, or -1 when not selected
    if (j >= 0) v = zsrc[j * zstride + col];
  }
  if constexpr (sizeof(OUT) == 2) {
    float rest = (float)v;  // the FP32 split of the layout notes above
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const __hip_bfloat16 part = __float2bfloat16(rest);
      out[p * total + idx] = part;
      rest -= __bfloat162float(part);
    }
  } else {
    out[idx] = (OUT)v;
  }
}

// One column tile: Z64 points at the tile's first column, k is the tile's
// width and zstride the row stride of Z64 (the full k).
template <typename OUT, int EL, int NP>
__global__ void pack_z_kernel(int64_t d, int64_t k, const int32_t* __restrict__ inv_perm,
                              const double* __restrict__ Z64, int64_t zstride, OUT* __restrict__ out, int64_t nt,
                              int64_t cbn) {
  const int total = (int)(nt * cbn * 64 * EL);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  pack_element<OUT, EL, NP>(idx, total, (int)d, (int)k, (int)cbn, inv_perm, Z64, (int)zstride, out);
}

// CSR operand value of element idx of the d x 64 row-major Z_full.
template <typename OUT>
__device__ __forceinline__ void pack_rowmajor_element(int idx, int k, const int32_t* inv, const double* zsrc,
                                                      int zstride, OUT* out) {
  const int row = idx / 64, col = idx % 64;
  double v = 0.0;
  if (col < k) {
    const int32_t j = inv[row];
    if (j >= 0) v = zsrc[j * zstride + col];
  }
  out[idx] = (OUT)v;
}

// inv_perm[c] = pivot position of column c (-1 when c is not among the r
// selected columns).
__global__ void inverse_perm_kernel(int64_t d, const int32_t* __restrict__ perm, const int64_t* __restrict__ rank,
                                    int32_t* __restrict__ inv_perm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const int64_t r = *rank;
  inv_perm[perm[j]] = j < r ? (int32_t)j : -1;
}

// CSR operand: Z_full row-major with rows padded to 64 columns.
template <typename OUT>
__global__ void pack_z_rowmajor_kernel(int64_t d, int64_t k, const int32_t* __restrict__ inv_perm,
                                       const double* __restrict__ Z64, int64_t zstride, OUT* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * 64) return;
  pack_rowmajor_element<OUT>(idx, (int)k, inv_perm, Z64, (int)zstride, out);
}

constexpr int64_t chunk_cols(int variant) { return variant == 0 ? 8 : (variant == 1 ? 16 : 32); }
constexpr int parts(int variant) { return variant == 3 ? 2 : (variant == 4 ? 3 : 1); }

// Z = R11^{-1} G_k and its pass-2 operand in one workgroup (r <= 256,
// k <= 64): the blocked solve above, then Z and the operand from LDS.
template <int VARIANT, int KB>
__global__ __launch_bounds__(1024) void form_z_kernel(int64_t d, int64_t k, const double* __restrict__ R,
                                                      const int64_t* __restrict__ rank,
                                                      const int32_t* __restrict__ perm,
                                                      const double* __restrict__ Gk, double* __restrict__ Z64,
                                                      void* __restrict__ Zpack, int64_t nt, int64_t cbn,
                                                      int32_t* err) {
  __shared__ double lds[kSolveLdsDoubles];
  __shared__ int32_t ready[16];
  __shared__ int32_t inv[kTrsmR];
  using F = PackForm<VARIANT>;
  const int r = (int)*rank, di = (int)d;
  for (int j = threadIdx.x; j < di; j += 1024) inv[perm[j]] = j < r ? j : -1;
  blocked_solve<KB>(lds, ready, di, (int)k, 0, R, r, Gk, err);  // ends with a barrier: inv is visible
  store_z64<KB>(lds, di, (int)k, 0, r, Z64);
  const int total = F::kRowMajor ? di * 64 : (int)(nt * cbn * 64 * F::EL);
  store_operand<VARIANT, KB>(lds, inv, di, total, Zpack);
}

// The update between diagonal blocks: G[0:j0, :] -= R[0:j0, j0:j0+kb] Z_q,
// Z_q = Z64[j0:j0+kb, :] (kb <= 256).  A tiled GEMM of this shape (a few
// hundred rows, k <= 64 columns) has only a dozen workgroups, so here each
// workgroup owns one 16 x 16 block of G and its four waves split the
// contraction in quarters of at most 64 (16 FP64 MFMA steps each, operands
// loaded straight into registers, no LDS staging); the quarters are added
// in wave order through LDS and the sum subtracted from G.
constexpr int kUpdK = kTrsmR / 4;  // contraction quarter per wave

__global__ __launch_bounds__(256) void trsm_update_kernel(int64_t j0, int64_t kb, int64_t d, int64_t k,
                                                          const double* __restrict__ R,
                                                          const double* __restrict__ Z64,
                                                          double* __restrict__ G) {
  __shared__ double part[3][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.y * 16, n0 = (int64_t)blockIdx.x * 16;
  // step s of this wave: contraction index kk = wave * kUpdK + 4 s + g; lane
  // l supplies A[l % 16][l / 16] = R[m0 + i][j0 + kk] and B[l / 16][l % 16] =
  // Z_q[kk][n0 + i] (zero past the block, the rows or the columns)
  const int64_t row = m0 + i, col = n0 + i;
  double av[kUpdK / 4], bv[kUpdK / 4];
#pragma unroll
  for (int st = 0; st < kUpdK / 4; ++st) {
    const int64_t kk = (int64_t)wave * kUpdK + 4 * st + g;
    const bool in_k = kk < kb;
    av[st] = (in_k && row < j0) ? R[row * d + j0 + kk] : 0.0;
    bv[st] = (in_k && col < k) ? Z64[(j0 + kk) * k + col] : 0.0;
  }
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < kUpdK / 4; ++st) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bv[st], acc, 0, 0, 0);
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wave - 1][v][lane] = acc[v];
  }
  __syncthreads();
  if (wave != 0) return;
  // accumulator element v of lane l: row g + 4 v, column i of the block
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double sum = ((acc[v] + part[0][v][lane]) + part[1][v][lane]) + part[2][v][lane];
    const int64_t r = m0 + g + 4 * v;
    if (r < j0 && col < k) G[r * k + col] -= sum;
  }
}

}  // namespace

hipError_t launch_trsm_z(int64_t d, int64_t k, const double* R, const int64_t* rank, double* G, double* Z64,
                         int32_t* err, hipStream_t s) {
  if (d <= 0 || k <= 0) return hipSuccess;
  // Blocked back substitution over diagonal blocks of 256 pivot positions,
  // last block first: solve block q, then subtract its contribution
  // R[0:j0, j0:j0+256] Z_q from the right-hand side of every row above it.
  // The block bounds do not depend on the rank (it stays on the device): Z
  // rows past the rank are exact zeros, so an update from a block past the
  // rank changes nothing in the rows that are solved.
  const dim3 grid(1, (unsigned)((k + 63) / 64));
  for (int64_t j0 = ((d - 1) / kTrsmR) * kTrsmR; j0 >= 0; j0 -= kTrsmR) {
    trsm_blocked_kernel<<<grid, 1024, 0, s>>>(d, k, j0, R, rank, G, Z64, err);
    if (j0 > 0) {
      const int64_t kb = std::min<int64_t>(kTrsmR, d - j0);
      const dim3 ugrid((unsigned)((k + 15) / 16), (unsigned)((j0 + 15) / 16));
      trsm_update_kernel<<<ugrid, 256, 0, s>>>(j0, kb, d, k, R, Z64, G);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

namespace {

// Bytes of one packed column tile of width kt <= 64.
size_t pack_tile_bytes(int variant, int64_t d, int64_t kt) {
  if (variant == 5 || variant == 6) return (size_t)d * 64 * (variant == 5 ? 4 : 8);
  if (variant < 0 || variant > 4) return 0;
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (kt + 15) / 16;
  const int64_t elems = nt * cbn * 64 * (cw / 4);
  const size_t esize = variant == 0 ? 8 : (variant == 1 ? 4 : 2);
  return (size_t)elems * esize * (size_t)parts(variant);
}

hipError_t pack_tile(int variant, int64_t d, int64_t kt, const int32_t* inv, const double* Z64, int64_t zstride,
                     void* out, hipStream_t s) {
  if (variant == 5 || variant == 6) {
    const unsigned blocks = (unsigned)((d * 64 + 255) / 256);
    if (variant == 5)
      pack_z_rowmajor_kernel<float><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<float*>(out));
    else
      pack_z_rowmajor_kernel<double><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<double*>(out));
    return hipGetLastError();
  }
  const int64_t cw = chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (kt + 15) / 16;
  const int64_t total = nt * cbn * 64 * (cw / 4);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  using bf = __hip_bfloat16;
  switch (variant) {
    case 0:
      pack_z_kernel<double, 2, 1><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<double*>(out), nt, cbn);
      break;
    case 1:
      pack_z_kernel<float, 4, 1><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<float*>(out), nt, cbn);
      break;
    case 2:
      pack_z_kernel<bf, 8, 1><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<bf*>(out), nt, cbn);
      break;
    case 3:
      pack_z_kernel<bf, 8, 2><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<bf*>(out), nt, cbn);
      break;
    case 4:
      pack_z_kernel<bf, 8, 3><<<blocks, 256, 0, s>>>(d, kt, inv, Z64, zstride, static_cast<bf*>(out), nt, cbn);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t pack_z_tile_offset(int variant, int64_t d, int64_t k, int64_t t) {
  (void)k;
  return (size_t)t * pack_tile_bytes(variant, d, kZTile);  // every tile before the last is full
}

size_t pack_z_operand_bytes(int variant, int64_t d, int64_t k) {
  if (variant < 0 || variant > 6 || k <= 0) return 0;
  const int64_t last = k - (z_tiles(k) - 1) * kZTile;
  return pack_z_tile_offset(variant, d, k, z_tiles(k) - 1) + pack_tile_bytes(variant, d, last);
}

size_t pack_z_bytes(int variant, int64_t d, int64_t k) {
  if (variant < 0 || variant > 6) return 0;
  return pack_z_operand_bytes(variant, d, k) + (size_t)d * sizeof(int32_t);
}

// Zpack layout: the packed operand (its column tiles in order) followed by
// inv_perm[d].
hipError_t launch_pack_z(int variant, int64_t d, int64_t k, const int32_t* perm, const int64_t* rank,
                         const double* Z64, void* Zpack, hipStream_t s) {
  if (variant < 0 || variant > 6) return hipErrorInvalidValue;
  char* base = static_cast<char*>(Zpack);
  int32_t* inv = reinterpret_cast<int32_t*>(base + pack_z_operand_bytes(variant, d, k));
  inverse_perm_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, perm, rank, inv);
  for (int64_t t = 0; t < z_tiles(k); ++t) {
    const int64_t c0 = t * kZTile, kt = std::min<int64_t>(kZTile, k - c0);
    hipError_t e = pack_tile(variant, d, kt, inv, Z64 + c0, k, base + pack_z_tile_offset(variant, d, k, t), s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_form_z(int variant, int64_t d, int64_t k, const double* R, const int64_t* rank,
                         const int32_t* perm, double* Gk, double* Z64, void* Zpack, int32_t* err,
                         hipStream_t s) {
  if (variant < 0 || variant > 6) return hipErrorInvalidValue;
  if (d > kTrsmR || k > 64) {
    hipError_t e = launch_trsm_z(d, k, R, rank, Gk, Z64, err, s);
    if (e != hipSuccess) return e;
    return launch_pack_z(variant, d, k, perm, rank, Z64, Zpack, s);
  }
  const int64_t cw = variant >= 5 ? 1 : chunk_cols(variant);
  const int64_t nt = (d + cw - 1) / cw;
  const int64_t cbn = (k + 15) / 16;
#define LEV_FZ(V)                                                                                      \
  case V:                                                                                              \
    switch (cbn) {                                                                                     \
      case 1: form_z_kernel<V, 1><<<1, 1024, 0, s>>>(d, k, R, rank, perm, Gk, Z64, Zpack, nt, cbn, err); break; \
      case 2: form_z_kernel<V, 2><<<1, 1024, 0, s>>>(d, k, R, rank, perm, Gk, Z64, Zpack, nt, cbn, err); break; \
      case 3: form_z_kernel<V, 3><<<1, 1024, 0, s>>>(d, k, R, rank, perm, Gk, Z64, Zpack, nt, cbn, err); break; \
      default: form_z_kernel<V, 4><<<1, 1024, 0, s>>>(d, k, R, rank, perm, Gk, Z64, Zpack, nt, cbn, err); break; \
    }                                                                                                  \
    break;
  switch (variant) {
    LEV_FZ(0) LEV_FZ(1) LEV_FZ(2) LEV_FZ(3) LEV_FZ(4) LEV_FZ(5) LEV_FZ(6)
  }
#undef LEV_FZ
  return hipGetLastError();
}

}  // namespace lev
