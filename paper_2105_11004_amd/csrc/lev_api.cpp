// C interface of liblev (declarations and contracts in include/lev.h):
// argument validation, seed expansion, workspace carving and the launch
// sequence of Algorithm 10 (LS-HRN-approx) = Algorithm 4 + Algorithm 8.
#include "lev.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "lev_internal.h"

namespace {

thread_local std::string g_last_error;

// Workspace of lev_estimate_noalloc: one copy per GPU, held from the first
// call on that GPU until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns for
// the current device, cached per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local hipEvent_t g_phase_events[LEV_PHASES];
thread_local bool g_phase_on = false;

hipError_t mark_phase(int i, hipStream_t s) {
  return g_phase_on ? hipEventRecord(g_phase_events[i], s) : hipSuccess;
}

lev_status fail(lev_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

lev_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(LEV_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LEV_OK;
}

#define LEV_TRY(expr)                          \
  do {                                         \
    lev_status _st = (expr);                   \
    if (_st != LEV_OK) return _st;             \
  } while (0)

#define LEV_HIP(expr) LEV_TRY(hip_check((expr), #expr))

// ---- seed expansion (SplitMix64, Steele-Lea-Flood 2014) --------------------
uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool is_prime_u64(uint64_t x) {
  if (x < 2) return false;
  if (x % 2 == 0) return x == 2;
  for (uint64_t f = 3; f * f <= x; f += 2)
    if (x % f == 0) return false;
  return true;
}

uint64_t next_prime_u64(uint64_t x) {
  uint64_t p = x < 2 ? 2 : x;
  while (!is_prime_u64(p)) ++p;
  return p;
}

// a^{-1} mod p (p prime, 0 < a < p), extended Euclid.
uint64_t modinv(uint64_t a, uint64_t p) {
  int64_t t = 0, new_t = 1;
  int64_t r = (int64_t)p, new_r = (int64_t)a;
  while (new_r != 0) {
    const int64_t q = r / new_r;
    int64_t tmp = t - q * new_t;
    t = new_t;
    new_t = tmp;
    tmp = r - q * new_r;
    r = new_r;
    new_r = tmp;
  }
  if (t < 0) t += (int64_t)p;
  return (uint64_t)t;
}

constexpr uint64_t kP61 = (1ull << 61) - 1;
// Rank cutoffs.  The Gram pivoting alone decides ranks reliably only while
// R_jj / R_00 stays far above sqrt(u) ~ 1.5e-8 (the Gram is rounded at
// u R_00^2): it is used alone for zeta >= kZetaGram.  Below that the refined
// path (rrqr.hip) resolves cutoffs down to kZetaMin, the FP64 cutoff of the
// paper's experiments; smaller cutoffs are refused.
constexpr double kZetaGram = 1e-5;
constexpr double kZetaMin = 1e-10;
constexpr int64_t kMaxRows = (1ll << 31) - 2;  // row ids + sign bit in 32 bits
constexpr int64_t kMaxD = 1024;
constexpr int64_t kMaxK = 4096;    // JL columns (pass 2 runs one pass per 64)
constexpr int64_t kMaxBwdK = 64;  // the backward's register tiles
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace (or a sizing pass when base is null).
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += align_up(count * sizeof(T));
    return p;
  }
};

size_t elem_size(int dtype) {
  switch (dtype) {
    case LEV_F64: return 8;
    case LEV_F32: return 4;
    case LEV_BF16: return 2;
    default: return 0;
  }
}

// pass-2 variant from the format, the storage type and the requested precision
int az_variant(int format, int dtype, int az) {
  if (format == LEV_CSR) {
    // CSR pass 2 runs on the vector ALUs: FP64 for F64 values, else FP32
    if (dtype == LEV_F64) return az == LEV_AZ_NATIVE ? 6 : -1;
    return (az == LEV_AZ_NATIVE || az == LEV_AZ_FP32) ? 5 : -1;
  }
  if (dtype == LEV_F64) return az == LEV_AZ_NATIVE ? 0 : -1;
  if (dtype == LEV_F32) {
    if (az == LEV_AZ_NATIVE || az == LEV_AZ_BF16X3) return 4;
    return az == LEV_AZ_FP32 ? 1 : -1;
  }
  if (dtype == LEV_BF16) {
    switch (az) {
      case LEV_AZ_NATIVE: return 2;
      case LEV_AZ_FP32: return 1;
      case LEV_AZ_BF16: return 2;
      case LEV_AZ_BF16X2: return 3;
      case LEV_AZ_BF16X3: return 4;  // Z in three BF16 parts (A is exact in BF16)
      default: return -1;
    }
  }
  return -1;
}

lev_status check_matrix(const lev_matrix* A) {
  if (A == nullptr) return fail(LEV_ERR_ARG, "A is null");
  if (A->format != LEV_DENSE_ROWMAJOR && A->format != LEV_CSR)
    return fail(LEV_ERR_ARG, "unknown format %d", A->format);
  if (elem_size(A->dtype) == 0) return fail(LEV_ERR_DTYPE, "unknown dtype %d", A->dtype);
  if (A->n < 0 || A->n > kMaxRows) return fail(LEV_ERR_SHAPE, "n = %lld out of range", (long long)A->n);
  if (A->d < 1 || A->d > kMaxD)
    return fail(LEV_ERR_SHAPE, "d = %lld outside [1, %lld]", (long long)A->d, (long long)kMaxD);
  if (A->format == LEV_DENSE_ROWMAJOR) {
    if (A->ld < A->d) return fail(LEV_ERR_SHAPE, "ld = %lld < d", (long long)A->ld);
    if (A->n > 0 && A->values == nullptr) return fail(LEV_ERR_ARG, "A->values is null");
    if ((reinterpret_cast<uintptr_t>(A->values) & 15) != 0)
      return fail(LEV_ERR_ARG, "A->values must be 16-byte aligned");
    if ((A->ld * (int64_t)elem_size(A->dtype)) % 16 != 0)
      return fail(LEV_ERR_ARG, "ld * sizeof(element) must be a multiple of 16 bytes");
  } else {
    if (A->nnz < 0) return fail(LEV_ERR_SHAPE, "nnz = %lld < 0", (long long)A->nnz);
    if (A->row_ptr == nullptr) return fail(LEV_ERR_ARG, "A->row_ptr is null");
    if (A->nnz > 0 && (A->col_idx == nullptr || A->values == nullptr))
      return fail(LEV_ERR_ARG, "A->col_idx or A->values is null");
  }
  return LEV_OK;
}

// uses_zeta: false for lev_sketch, which takes no rank decision.
lev_status check_params(const lev_matrix* A, const lev_params* p, bool uses_zeta = true) {
  if (p == nullptr) return fail(LEV_ERR_ARG, "params is null");
  if (p->r_cs < 1 || p->r_cs > kMaxRows) return fail(LEV_ERR_ARG, "r_cs = %lld out of range", (long long)p->r_cs);
  const bool sketched = p->mode != LEV_MODE_QLESS;  // Algorithm 6 takes no sketch: m and sketch unused
  if (sketched && p->m < A->d) return fail(LEV_ERR_SHAPE, "m = %lld < d = %lld", (long long)p->m, (long long)A->d);
  if (p->m > (1ll << 24)) return fail(LEV_ERR_SHAPE, "m too large");
  if (p->mode != LEV_MODE_JL && p->mode != LEV_MODE_EXACT && p->mode != LEV_MODE_NOJL && p->mode != LEV_MODE_QLESS)
    return fail(LEV_ERR_ARG, "mode %d is not one of the LEV_MODE_* values", p->mode);
  if (p->mode == LEV_MODE_QLESS) {
    if (p->k < 1) return fail(LEV_ERR_ARG, "k (the step cap of the Q-less QR) must be >= 1");
    if (uses_zeta && p->zeta < kZetaGram)
      return fail(LEV_ERR_NOT_SUPPORTED, "the Q-less QR decides its rank from downdated norms: zeta >= %g", kZetaGram);
  }
  if (p->sketch != LEV_SKETCH_GAUSS && p->sketch != LEV_SKETCH_SRHT)
    return fail(LEV_ERR_ARG, "sketch %d is not LEV_SKETCH_GAUSS or LEV_SKETCH_SRHT", p->sketch);
  if (sketched && p->sketch == LEV_SKETCH_SRHT) {
    if ((p->r_cs & (p->r_cs - 1)) != 0)
      return fail(LEV_ERR_ARG, "the SRHT needs r_cs a power of two (r_cs = %lld)", (long long)p->r_cs);
    if (p->m > p->r_cs)
      return fail(LEV_ERR_SHAPE, "the SRHT samples m <= r_cs rows (m = %lld)", (long long)p->m);
  }
  if (p->mode == LEV_MODE_JL && (p->k < 1 || p->k > kMaxK))
    return fail(LEV_ERR_ARG, "k = %lld outside [1, %lld]", (long long)p->k, (long long)kMaxK);
  if (!(p->zeta >= 0.0 && p->zeta < 1.0)) return fail(LEV_ERR_ARG, "zeta must be in [0, 1)");
  if (uses_zeta && p->zeta < kZetaMin)
    return fail(LEV_ERR_NOT_SUPPORTED, "zeta = %g is below the smallest supported rank cutoff %g", p->zeta, kZetaMin);
  if (az_variant(A->format, A->dtype, p->az_precision) < 0)
    return fail(LEV_ERR_ARG, "az_precision %d not valid for dtype %d", p->az_precision, A->dtype);
  return LEV_OK;
}

// Columns of the pass-2 operand Z: the JL columns k, or (no JL step, exact
// scores) all d columns of R11^{-1}, of which the first r can be nonzero.
int64_t pass2_cols(const lev_matrix* A, const lev_params* p) { return p->mode == LEV_MODE_JL ? p->k : A->d; }

lev_status check_ws(const void* ws, size_t have, size_t need) {
  if (need > have) return fail(LEV_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", have, need);
  if (need > 0 && ws == nullptr) return fail(LEV_ERR_WORKSPACE, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0)
    return fail(LEV_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return LEV_OK;
}

// ---- state blob ---------------------------------------------------------------
struct StateView {
  int64_t* header;  // [0] magic, [1] d, [2] m, [3] k, [4] rank, [5] error word (low 32 bits)
  int32_t* perm;
  double* R;
  double* Z64;
  double* At;
};
constexpr int64_t kStateMagic = 0x4C45565354415431ll;

size_t state_bytes(int64_t d, int64_t m, int64_t k) {
  Carver c(nullptr);
  c.take<int64_t>(8);
  c.take<int32_t>((size_t)d);
  c.take<double>((size_t)(d * d));
  c.take<double>((size_t)(d * k));
  c.take<double>((size_t)(m * d));
  return c.used;
}

StateView carve_state(void* base, int64_t d, int64_t m, int64_t k) {
  Carver c(base);
  StateView v;
  v.header = c.take<int64_t>(8);
  v.perm = c.take<int32_t>((size_t)d);
  v.R = c.take<double>((size_t)(d * d));
  v.Z64 = c.take<double>((size_t)(d * k));
  v.At = c.take<double>((size_t)(m * d));
  return v;
}

// The device error word of a state blob (bits lev::kErrPivotWait,
// lev::kErrSolveWait).
int32_t* state_err(const StateView& v) { return reinterpret_cast<int32_t*>(v.header + 5); }

// ---- workspace plans -------------------------------------------------------------
struct SketchBufs {
  double* Gm;        // FP64 G_m (m x r_cs), or null when x3 or SRHT
  double* SA;
  double* partial;
  bool x3 = false;   // the transform in FP32-level arithmetic (xgemm.hip)
  uint32_t* Gp;      // x3: G_m as three BF16 parts
  void* SAp;         // x3: (S A)^T as three BF16 parts
  bool srht = false; // A~ = F (S A) with the SRHT F (srht.hip) instead of G_m
  int32_t* inv;      // SRHT: the sampled coordinates (r_cs)
};

int gm_splits(int64_t m, int64_t d, int64_t r_cs) { return lev::dgemm_choose_splits(m, d, r_cs); }

// The Gaussian transform runs in FP32-level arithmetic on the BF16 matrix
// cores (six products of three-part splits) for BF16-stored dense A, whose
// entries carry 8 significant bits: its relative error ~2^-24 is far below
// them, and the FP64 product would take longer than either pass over A.
// Every other input keeps the FP64 transform.
bool use_x3_transform(const lev_matrix* A, int64_t r_cs) {
  return A->format == LEV_DENSE_ROWMAJOR && A->dtype == LEV_BF16 && r_cs % 8 == 0;
}

SketchBufs carve_sketch_bufs(Carver& c, int64_t d, int64_t m, int64_t r_cs, bool need_sa, bool x3) {
  SketchBufs b;
  b.x3 = x3;
  if (x3) {
    b.Gm = nullptr;
    b.Gp = c.take<uint32_t>(3 * lev::split3_elems(m, r_cs) / 2);
    b.SAp = c.take<uint32_t>(3 * lev::split3_elems(d, r_cs) / 2);
    b.SA = c.take<double>((size_t)(r_cs * d));
    b.partial = c.take<double>(lev::xgemm_partial_elems(m, d, lev::xgemm_choose_splits(m, d, r_cs)));
    return b;
  }
  b.Gp = nullptr;
  b.SAp = nullptr;
  b.Gm = c.take<double>((size_t)(m * r_cs));
  b.SA = need_sa ? c.take<double>((size_t)(r_cs * d)) : nullptr;
  b.partial = c.take<double>(lev::dgemm_partial_elems(m, d, gm_splits(m, d, r_cs)));
  return b;
}

// The sketch's buffers for A and p: the SRHT needs S A (transformed in
// place) and the sample map; the Gaussian stage G_m (FP64, or its three BF16
// parts for the FP32-level transform) and the product's partial sums.
SketchBufs carve_sketch(Carver& c, const lev_matrix* A, const lev_params* p) {
  if (p->sketch == LEV_SKETCH_SRHT) {
    SketchBufs b;
    b.srht = true;
    b.Gm = nullptr;
    b.partial = nullptr;
    b.Gp = nullptr;
    b.SAp = nullptr;
    b.SA = c.take<double>((size_t)(p->r_cs * A->d));
    b.inv = c.take<int32_t>((size_t)p->r_cs);
    return b;
  }
  return carve_sketch_bufs(c, A->d, p->m, p->r_cs, true, use_x3_transform(A, p->r_cs));
}

struct RankBufs {
  double* B;
  double* partial;
  lev::PivCholState pc;
};

RankBufs carve_rank(Carver& c, int64_t m, int64_t d) {
  RankBufs b;
  b.B = c.take<double>((size_t)(d * d));
  b.partial = c.take<double>(lev::dgemm_partial_elems(d, d, lev::gram_sketch_splits(m, d)));
  b.pc.diag = c.take<double>((size_t)d);
  b.pc.Rrows = c.take<double>((size_t)(d * d));
  b.pc.piv = c.take<int32_t>((size_t)d);
  b.pc.flags = c.take<int32_t>(64);
  b.pc.r00 = c.take<double>(1);
  b.pc.err = nullptr;
  return b;
}

// Buffers of the refined rank-revealing path (zeta < kZetaGram).
struct RefineBufs {
  double *X1, *X2, *Qa, *Q;                        // m x d
  double *I, *Rinv, *Bq, *W1, *W2, *Rtop, *Rbot;  // d x d
  double *R1, *Rf, *R2;                            // d x d
  int32_t *perm1, *permf, *perm2;                  // d
  int64_t *r1, *rf, *r2;                           // device scalars
  lev::PivCholState stf, st2;
  double* partial;
};

lev::PivCholState carve_pivchol_state(Carver& c, int64_t d) {
  lev::PivCholState st;
  st.diag = c.take<double>((size_t)d);
  st.Rrows = c.take<double>((size_t)(d * d));
  st.piv = c.take<int32_t>((size_t)d);
  st.flags = c.take<int32_t>(64);
  st.r00 = c.take<double>(1);
  st.err = nullptr;
  return st;
}

RefineBufs carve_refine(Carver& c, int64_t m, int64_t d) {
  RefineBufs b;
  double** md[] = {&b.X1, &b.X2, &b.Qa, &b.Q};
  for (double** p : md) *p = c.take<double>((size_t)(m * d));
  double** dd[] = {&b.I, &b.Rinv, &b.Bq, &b.W1, &b.W2, &b.Rtop, &b.Rbot, &b.R1, &b.Rf, &b.R2};
  for (double** p : dd) *p = c.take<double>((size_t)(d * d));
  b.perm1 = c.take<int32_t>((size_t)d);
  b.permf = c.take<int32_t>((size_t)d);
  b.perm2 = c.take<int32_t>((size_t)d);
  b.r1 = c.take<int64_t>(1);
  b.rf = c.take<int64_t>(1);
  b.r2 = c.take<int64_t>(1);
  b.stf = carve_pivchol_state(c, d);
  b.st2 = carve_pivchol_state(c, d);
  size_t mx = 0;
  const int64_t shapes[2][3] = {{m, d, d}, {d, d, m}};
  for (const auto& sh : shapes)
    mx = std::max(mx, lev::dgemm_partial_elems(sh[0], sh[1], lev::dgemm_choose_splits(sh[0], sh[1], sh[2])));
  b.partial = c.take<double>(mx);
  return b;
}

// Gk (d x k, may be null): the JL Gaussian, drawn alongside G_m.
lev_status enqueue_sketch(const lev_matrix* A, const lev_params* p, const lev::SeedDraws& dr,
                          const SketchBufs& b, double* SA, double* At, double* Gk, hipStream_t s) {
  const int64_t d = A->d, m = p->m, r_cs = p->r_cs, k = p->k;
  // G_m and G_k are drawn by pass 1's workgroups (compute under its memory traffic)
  lev::GaussDraw g{{{dr.key_m, m * r_cs, 1.0 / std::sqrt((double)m), b.Gm},
                    {dr.key_k, d * k, 1.0 / std::sqrt((double)k), Gk}}};
  if (b.x3) g.m[0].parts3 = b.Gp;  // G_m drawn straight into its three parts
  if (b.srht) g.m[0].total = 0;     // no G_m
  // the split-form transform reads S A only through its FP32 value: pass 1
  // stores it as float (in the internal buffer; a caller's SA_out keeps FP64)
  const bool sa32 = b.x3 && SA == b.SA && A->n > 0 && A->format != LEV_CSR;
  void* sa_buf = SA;
  LEV_HIP(mark_phase(1, s));
  if (A->n > 0 && A->format == LEV_CSR) {
    LEV_HIP(lev::launch_countsketch_csr(A->dtype, A->values, A->row_ptr, A->col_idx, A->n, d, A->nnz, dr.hash,
                                        SA, g, s));
  } else if (A->n > 0) {
    LEV_HIP(lev::launch_countsketch_dense(A->dtype, A->values, A->n, d, A->ld, dr.hash, sa_buf, sa32, g, s));
  } else {
    if (!b.x3 && !b.srht) LEV_HIP(lev::launch_gaussian(dr.key_m, m, r_cs, g.m[0].scale, b.Gm, s));
    if (Gk != nullptr) LEV_HIP(lev::launch_gaussian(dr.key_k, d, k, g.m[1].scale, Gk, s));
    LEV_HIP(lev::launch_fill_zero(SA, sizeof(double) * (size_t)(r_cs * d), s));
  }
  LEV_HIP(mark_phase(2, s));
  // A~ = G_m (S A): (m x r_cs) (r_cs x d), or F (S A) with the SRHT F
  if (b.srht) {
    if (SA != b.SA)
      LEV_HIP(hipMemcpyAsync(b.SA, SA, sizeof(double) * (size_t)(r_cs * d), hipMemcpyDeviceToDevice, s));
    LEV_HIP(lev::launch_srht(dr.key_d, dr.key_p, r_cs, d, m, b.SA, b.inv, At, s));
  } else if (b.x3 && A->n > 0) {
    LEV_HIP(lev::launch_split_t3(r_cs, d, sa_buf, sa32, b.SAp, s));
    LEV_HIP(lev::launch_xgemm(m, d, r_cs, b.Gp, b.SAp, At, d, lev::xgemm_choose_splits(m, d, r_cs), b.partial, s));
  } else if (b.x3) {
    LEV_HIP(lev::launch_fill_zero(At, sizeof(double) * (size_t)(m * d), s));
  } else {
    const int splits = gm_splits(m, d, r_cs);
    LEV_HIP(lev::launch_dgemm(m, d, r_cs, 1.0, b.Gm, r_cs, 1, SA, d, 1, 0.0, At, d, splits, b.partial,
                              nullptr, s));
  }
  LEV_HIP(mark_phase(3, s));
  return LEV_OK;
}

// C = op(A) op(B) (beta = 0) or C += alpha op(A) op(B) (beta = 1) with the
// split the shape calls for; strides as in launch_dgemm.
lev_status gemm_ab(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sai, int64_t sak,
                   const double* B, int64_t sbk, int64_t sbj, double beta, double* C, double* partial,
                   hipStream_t s) {
  const int sp = lev::dgemm_choose_splits(M, N, K);
  return hip_check(lev::launch_dgemm(M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, N, sp, partial, nullptr, s),
                   "dgemm");
}

// Pivoted Cholesky of B (d x d, overwritten) into st, then perm / R / rank.
lev_status pivchol_into(double* B, int64_t d, double zeta, const lev::PivCholState& st, int64_t* rank,
                        int32_t* perm, double* R, double* partial, hipStream_t s, int fixed = 0,
                        const double* ref_r00 = nullptr) {
  // the panel path (d > 256) tracks progress in flags; the single-workgroup
  // path does not read them
  if (d > 256) LEV_HIP(lev::launch_fill_zero(st.flags, 64 * sizeof(int32_t), s));
  LEV_HIP(lev::launch_pivchol(B, d, zeta, st, rank, partial, s, fixed, ref_r00));
  LEV_HIP(lev::launch_pivchol_finalize(d, st, rank, perm, R, s));
  return LEV_OK;
}

// Q (m x d) = an orthonormal basis of the first r columns of X (the other
// columns of X and Q zero) by Cholesky QR twice, starting from the Cholesky
// factor Rc of X^T X that the pivoting already produced (rows < r): Qa =
// X Rc^{-1}, then Qa^T Qa = Rf^T Rf (plain Cholesky, fixed order) and Q =
// Qa Rf^{-1}.  One pass leaves Qa^T Qa - I at about u kappa^2; the second
// brings it to rounding.
lev_status cholqr2(int64_t m, int64_t d, const double* X, const double* Rc, const int64_t* r, RefineBufs& b,
                   double* Q, int32_t* err, hipStream_t s) {
  LEV_HIP(lev::launch_identity(d, b.I, s));
  LEV_HIP(lev::launch_trsm_z(d, d, Rc, r, b.I, b.Rinv, err, s));  // Rc11^{-1}, zero past r
  LEV_TRY(gemm_ab(m, d, d, 1.0, X, d, 1, b.Rinv, d, 1, 0.0, b.Qa, b.partial, s));
  LEV_TRY(gemm_ab(d, d, m, 1.0, b.Qa, 1, d, b.Qa, d, 1, 0.0, b.Bq, b.partial, s));
  LEV_TRY(pivchol_into(b.Bq, d, 0.0, b.stf, b.rf, b.permf, b.Rf, b.partial, s, /*fixed=*/1));
  LEV_HIP(lev::launch_identity(d, b.I, s));
  LEV_HIP(lev::launch_trsm_z(d, d, b.Rf, b.rf, b.I, b.Rinv, err, s));
  LEV_TRY(gemm_ab(m, d, d, 1.0, b.Qa, d, 1, b.Rinv, d, 1, 0.0, Q, b.partial, s));
  return LEV_OK;
}

// Algorithm 4, steps 2-3: perm, R (sign-normalised, positive diagonal) and
// the cutoff rank of the column-pivoted QR of A~.  For zeta >= kZetaGram the
// pivoted Cholesky of the Gram decides alone; below it (rf != null) the
// refined path of rrqr.hip: stage 1 to kZetaGram, Cholesky QR twice of those
// columns, the rest projected off them twice, stage 2 on the residual's Gram
// with the cutoff zeta * R_00 of stage 1, Cholesky QR twice of the stage-2
// columns, R's rows as Q^T X.
lev_status enqueue_rank(const double* At, int64_t m, int64_t d, double zeta, const RankBufs& b,
                        int32_t* perm, double* R, int64_t* rank, hipStream_t s, RefineBufs* rf = nullptr) {
  // Gram B = A~^T A~ (d x d): the tiles on and above the diagonal, mirrored
  LEV_HIP(lev::launch_gram_dense(LEV_F64, At, m, d, d, lev::gram_sketch_splits(m, d), b.partial, b.B, s));
  if (zeta >= kZetaGram || rf == nullptr) return pivchol_into(b.B, d, zeta, b.pc, rank, perm, R, b.partial, s);

  RefineBufs& f = *rf;
  int32_t* err = b.pc.err;
  f.stf.err = err;
  f.st2.err = err;
  // stage 1: the columns the Gram resolves
  LEV_TRY(pivchol_into(b.B, d, kZetaGram, b.pc, f.r1, f.perm1, f.R1, b.partial, s));
  LEV_HIP(lev::launch_gather_split(m, d, f.perm1, f.r1, At, f.X1, f.X2, s));
  LEV_TRY(cholqr2(m, d, f.X1, f.R1, f.r1, f, f.Q, err, s));
  // the rest projected off range(Q1) twice; R's rows 0..r1-1 = Q1^T X
  LEV_TRY(gemm_ab(d, d, m, 1.0, f.Q, 1, d, f.X2, d, 1, 0.0, f.W1, f.partial, s));
  LEV_TRY(gemm_ab(m, d, d, -1.0, f.Q, d, 1, f.W1, d, 1, 1.0, f.X2, f.partial, s));
  LEV_TRY(gemm_ab(d, d, m, 1.0, f.Q, 1, d, f.X2, d, 1, 0.0, f.W2, f.partial, s));
  LEV_TRY(gemm_ab(m, d, d, -1.0, f.Q, d, 1, f.W2, d, 1, 1.0, f.X2, f.partial, s));
  LEV_TRY(gemm_ab(d, d, m, 1.0, f.Q, 1, d, f.X1, d, 1, 0.0, f.Rtop, f.partial, s));
  LEV_HIP(lev::launch_add2(d * d, f.Rtop, f.W1, f.W2, s));
  // stage 2: pivoting on the residual's Gram, cutoff zeta * R_00 of stage 1
  LEV_TRY(gemm_ab(d, d, m, 1.0, f.X2, 1, d, f.X2, d, 1, 0.0, f.Bq, f.partial, s));
  LEV_TRY(pivchol_into(f.Bq, d, zeta, f.st2, f.r2, f.perm2, f.R2, b.partial, s, 0, b.pc.r00));
  LEV_HIP(lev::launch_gather_split(m, d, f.perm2, f.r2, f.X2, f.X1, nullptr, s));  // X1 <- the stage-2 columns
  LEV_TRY(cholqr2(m, d, f.X1, f.R2, f.r2, f, f.Q, err, s));
  LEV_TRY(gemm_ab(d, d, m, 1.0, f.Q, 1, d, f.X2, d, 1, 0.0, f.Rbot, f.partial, s));
  LEV_HIP(lev::launch_rrqr_assemble(d, f.perm1, f.r1, f.perm2, f.r2, f.Rtop, f.Rbot, perm, R, rank, s));
  return LEV_OK;
}

// ---- backward plan ---------------------------------------------------------------
struct BwdBufs {
  void* Zpack;       // Z_full, variant 5/6 (d x 64 of the gradient's type) + inverse perm
  void* partials;    // groups x d x 64 elements
  double* C64;       // d x k
  double* Zbar;      // d x k
  double* sq[5];     // d x d scratch
  double* AtK;       // m x d
  double* Abar_t;    // m x d
  double* Gm;        // m x r_cs
  double* H;         // r_cs x d
  void* Hf;          // r_cs x d, gradient type
  double* gemm_partial;
  int groups;
};

size_t bwd_gemm_partial_elems(int64_t d, int64_t m, int64_t k, int64_t r_cs) {
  size_t mx = 0;
  const int64_t shapes[4][3] = {{d, d, k}, {d, d, d}, {m, d, d}, {r_cs, d, m}};
  for (const auto& sh : shapes) {
    const int sp = lev::dgemm_choose_splits(sh[0], sh[1], sh[2]);
    mx = std::max(mx, lev::dgemm_partial_elems(sh[0], sh[1], sp));
  }
  return mx;
}

BwdBufs carve_bwd(Carver& c, const lev_matrix* A, const lev_params* p) {
  const int64_t n = A->n, d = A->d, m = p->m, k = p->k, r_cs = p->r_cs;
  const int dt = A->dtype == LEV_F64 ? 0 : 1;
  const size_t es = lev::bwd_elem_size(dt);
  BwdBufs b;
  b.groups = lev::bwd_groups(dt, n, d, k);
  b.Zpack = c.take<char>(lev::pack_z_bytes(dt == 0 ? 6 : 5, d, k));
  b.partials = c.take<char>((size_t)b.groups * (size_t)d * 64 * es);
  b.C64 = c.take<double>((size_t)(d * k));
  b.Zbar = c.take<double>((size_t)(d * k));
  for (int i = 0; i < 5; ++i) b.sq[i] = c.take<double>((size_t)(d * d));
  b.AtK = c.take<double>((size_t)(m * d));
  b.Abar_t = c.take<double>((size_t)(m * d));
  b.Gm = c.take<double>((size_t)(m * r_cs));
  b.H = c.take<double>((size_t)(r_cs * d));
  b.Hf = c.take<char>((size_t)(r_cs * d) * es);
  b.gemm_partial = c.take<double>(bwd_gemm_partial_elems(d, m, k, r_cs));
  return b;
}

// LS-HRN-exact (Algorithm 7): B = A^T A and its partial sums, and a second
// pivoted Cholesky (of B_K) with its outputs.
struct ExactBufs {
  double* gram_partial;
  double* C64;
  RankBufs rb2;
  int32_t* perm2;
  double* R2;
  int64_t* rank2;
  int32_t* permc;
  double* I;
};

size_t gram_partial_elems(const lev_matrix* A) {
  if (A->format == LEV_CSR) return lev::gram_csr_partial_elems(A->n, A->d);
  return lev::dgemm_partial_elems(A->d, A->d, lev::gram_dense_splits(A->n, A->d));
}

ExactBufs carve_exact(Carver& c, const lev_matrix* A, const lev_params* p) {
  const int64_t d = A->d, m = p->m;
  ExactBufs b;
  b.gram_partial = c.take<double>(std::max<size_t>(1, gram_partial_elems(A)));
  b.C64 = c.take<double>((size_t)(d * d));
  b.rb2 = carve_rank(c, m, d);
  b.perm2 = c.take<int32_t>((size_t)d);
  b.R2 = c.take<double>((size_t)(d * d));
  b.rank2 = c.take<int64_t>(1);
  b.permc = c.take<int32_t>((size_t)d);
  b.I = c.take<double>((size_t)(d * d));
  return b;
}

lev_status check_backward_input(const lev_matrix* A, const lev_params* p) {
  if (p->mode != LEV_MODE_JL) return fail(LEV_ERR_NOT_SUPPORTED, "the backward pass is of the JL estimate only");
  if (p->sketch != LEV_SKETCH_GAUSS)
    return fail(LEV_ERR_NOT_SUPPORTED, "the backward pass takes the Gaussian sketch (LEV_SKETCH_GAUSS) only");
  if (p->k > kMaxBwdK)
    return fail(LEV_ERR_NOT_SUPPORTED, "the backward pass takes k <= %lld", (long long)kMaxBwdK);
  if (A->format != LEV_DENSE_ROWMAJOR)
    return fail(LEV_ERR_NOT_SUPPORTED, "the backward pass takes dense A only");
  if (A->dtype != LEV_F32 && A->dtype != LEV_F64)
    return fail(LEV_ERR_DTYPE, "the backward pass takes FP32 or FP64 A");
  return LEV_OK;
}

// C = alpha op(A) op(B) with the strides of launch_dgemm and the split the
// shape calls for.
lev_status gemm(int64_t M, int64_t N, int64_t K, const double* A, int64_t sai, int64_t sak, const double* B,
                int64_t sbk, int64_t sbj, double* C, double* partial, hipStream_t s) {
  const int sp = lev::dgemm_choose_splits(M, N, K);
  return hip_check(lev::launch_dgemm(M, N, K, 1.0, A, sai, sak, B, sbk, sbj, 0.0, C, N, sp, partial, nullptr, s),
                   "dgemm");
}

}  // namespace

namespace lev {

SeedDraws derive_draws(uint64_t seed, int64_t n, int64_t r_cs) {
  uint64_t st = seed;
  uint64_t w[10];
  for (int i = 0; i < 10; ++i) w[i] = splitmix64_next(st);
  SeedDraws dr;
  HashParams& h = dr.hash;
  h.n = n;
  h.r_cs = r_cs;
  h.P = next_prime_u64((uint64_t)(n < 2 ? 2 : n));
  h.a = 1 + w[0] % (h.P - 1);
  h.c = w[1] % h.P;
  h.ainv = modinv(h.a, h.P);
  h.delta = (h.ainv * ((uint64_t)r_cs % h.P)) % h.P;
  h.pbar = ~0ull / h.P;
  h.c0 = w[2] % kP61;
  h.c1 = w[3] % kP61;
  h.c2 = w[4] % kP61;
  h.c3 = w[5] % kP61;
  dr.key_m = PhiloxKey{(uint32_t)(w[6] & 0xFFFFFFFFu), (uint32_t)(w[6] >> 32)};
  dr.key_k = PhiloxKey{(uint32_t)(w[7] & 0xFFFFFFFFu), (uint32_t)(w[7] >> 32)};
  dr.key_d = w[8];
  dr.key_p = w[9];
  return dr;
}

}  // namespace lev

extern "C" {

const char* lev_status_string(lev_status s) {
  switch (s) {
    case LEV_OK: return "LEV_OK";
    case LEV_ERR_ARG: return "LEV_ERR_ARG";
    case LEV_ERR_SHAPE: return "LEV_ERR_SHAPE";
    case LEV_ERR_DTYPE: return "LEV_ERR_DTYPE";
    case LEV_ERR_FORMAT: return "LEV_ERR_FORMAT";
    case LEV_ERR_WORKSPACE: return "LEV_ERR_WORKSPACE";
    case LEV_ERR_HIP: return "LEV_ERR_HIP";
    case LEV_ERR_NOT_SUPPORTED: return "LEV_ERR_NOT_SUPPORTED";
    default: return "LEV_ERR_UNKNOWN";
  }
}

const char* lev_last_error(void) { return g_last_error.c_str(); }

lev_status lev_set_phase_events(hipEvent_t* events, int count) {
  if (events == nullptr || count == 0) {
    g_phase_on = false;
    return LEV_OK;
  }
  if (count != LEV_PHASES) return fail(LEV_ERR_ARG, "count must be %d", LEV_PHASES);
  for (int i = 0; i < LEV_PHASES; ++i) {
    if (events[i] == nullptr) return fail(LEV_ERR_ARG, "event %d is null", i);
    g_phase_events[i] = events[i];
  }
  g_phase_on = true;
  return LEV_OK;
}

size_t lev_state_size(int64_t d, int64_t m, int64_t k) {
  if (d < 1 || m < d || k < 1) return 0;
  return state_bytes(d, m, k);
}

size_t lev_rank_workspace_size(int64_t m, int64_t d) {
  if (d < 1 || d > kMaxD || m < d) return 0;
  Carver c(nullptr);
  carve_rank(c, m, d);
  carve_refine(c, m, d);  // any zeta: the size does not depend on it
  return c.used;
}

}  // extern "C"

namespace {  // helpers of the entry points below

// Algorithm 6: the Q-less pivoted QR of A (qless.hip), then Z = R_k^{-1}
// and pass 2 over the column tiles below the rank.
struct QlessBufs {
  double* qws;
  int32_t* perm;
  double* R;
  int64_t* rank;
  int32_t* err;
  double* I;
  double* Z64;
  void* Zpack;
};

int64_t qless_steps(const lev_matrix* A, const lev_params* p) { return std::min<int64_t>(p->k, A->d); }

QlessBufs carve_qless(Carver& c, const lev_matrix* A, const lev_params* p) {
  const int64_t d = A->d;
  QlessBufs b;
  b.qws = c.take<double>(lev::qless_ws_doubles(A->n, d, qless_steps(A, p), A->format == LEV_CSR));
  b.perm = c.take<int32_t>((size_t)d);
  b.R = c.take<double>((size_t)(d * d));
  b.rank = c.take<int64_t>(1);
  b.err = c.take<int32_t>(1);
  b.I = c.take<double>((size_t)(d * d));
  b.Z64 = c.take<double>((size_t)(d * d));
  b.Zpack = c.take<char>(lev::pack_z_bytes(az_variant(A->format, A->dtype, p->az_precision), d, d));
  return b;
}

}  // namespace

extern "C" {

size_t lev_workspace_size(const lev_matrix* A, const lev_params* p, int which) {
  if (check_matrix(A) != LEV_OK || check_params(A, p, which != LEV_WS_SKETCH) != LEV_OK) return 0;
  const int64_t d = A->d, m = p->m, k = p->k, r_cs = p->r_cs;
  Carver c(nullptr);
  if (which == LEV_WS_SKETCH) {
    carve_sketch(c, A, p);
    return c.used;
  }
  if (which == LEV_WS_ESTIMATE && p->mode == LEV_MODE_QLESS) {
    carve_qless(c, A, p);
    return c.used;
  }
  if (which == LEV_WS_ESTIMATE && p->mode == LEV_MODE_EXACT) {
    carve_sketch(c, A, p);
    carve_rank(c, m, d);
    if (p->zeta < kZetaGram) carve_refine(c, m, d);
    c.take<char>(state_bytes(d, m, d));
    carve_exact(c, A, p);
    c.take<char>(lev::pack_z_bytes(az_variant(A->format, A->dtype, p->az_precision), d, d));
    return c.used;
  }
  if (which == LEV_WS_ESTIMATE) {
    carve_sketch(c, A, p);
    carve_rank(c, m, d);
    if (p->zeta < kZetaGram) carve_refine(c, m, d);
    const int64_t kz = pass2_cols(A, p);
    c.take<char>(state_bytes(d, m, kz));
    c.take<double>((size_t)(d * kz));  // G_k (identity without the JL step)
    c.take<char>(lev::pack_z_bytes(az_variant(A->format, A->dtype, p->az_precision), d, kz));
    return c.used;
  }
  if (which == LEV_WS_BACKWARD) {
    if (check_backward_input(A, p) != LEV_OK) return 0;
    carve_bwd(c, A, p);
    return c.used;
  }
  return 0;
}

lev_status lev_sketch(const lev_matrix* A, const lev_params* p, double* At_out, double* SA_out, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  LEV_TRY(check_matrix(A));
  LEV_TRY(check_params(A, p, /*uses_zeta=*/false));
  if (At_out == nullptr) return fail(LEV_ERR_ARG, "At_out is null");
  Carver sizing(nullptr);
  carve_sketch(sizing, A, p);
  LEV_TRY(check_ws(ws, ws_bytes, sizing.used));
  Carver c(ws);
  SketchBufs b = carve_sketch(c, A, p);
  const lev::SeedDraws dr = lev::derive_draws(p->seed, A->n, p->r_cs);
  double* SA = SA_out != nullptr ? SA_out : b.SA;
  return enqueue_sketch(A, p, dr, b, SA, At_out, nullptr, stream);
}

lev_status lev_rank_estimate(const double* At, int64_t m, int64_t d, double zeta, int32_t* perm_out,
                             double* R_out, int64_t* rank_out, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (At == nullptr || perm_out == nullptr || R_out == nullptr || rank_out == nullptr)
    return fail(LEV_ERR_ARG, "null pointer argument");
  if (d < 1 || d > kMaxD) return fail(LEV_ERR_SHAPE, "d = %lld outside [1, 1024]", (long long)d);
  if (m < d) return fail(LEV_ERR_SHAPE, "m = %lld < d = %lld", (long long)m, (long long)d);
  if (!(zeta >= 0.0 && zeta < 1.0)) return fail(LEV_ERR_ARG, "zeta must be in [0, 1)");
  if (zeta < kZetaMin)
    return fail(LEV_ERR_NOT_SUPPORTED, "zeta = %g is below the smallest supported rank cutoff %g", zeta, kZetaMin);
  const size_t need = lev_rank_workspace_size(m, d);
  LEV_TRY(check_ws(ws, ws_bytes, need));
  Carver c(ws);
  RankBufs b = carve_rank(c, m, d);
  RefineBufs rf = carve_refine(c, m, d);
  return enqueue_rank(At, m, d, zeta, b, perm_out, R_out, rank_out, stream, &rf);
}

}  // extern "C"

namespace {  // helpers of the entry points below

// Algorithm 7 (LS-HRN-exact): the columns K and the rank from Algorithm 4
// on the sketch (as for Algorithm 10), then B = A^T A in one more pass over
// A (Algorithm 5's Gram route: FP64 matrix cores for dense A, sum_i nnz_i^2
// products for CSR), B_K = B[K, K], its pivoted Cholesky (A_K P2)^T (A_K P2)
// = R_B^T R_B, Z = R_B^{-1} and theta~_i = ||e_i^T A_K P2 R_B^{-1}||^2 in
// pass 2 over the column tiles of Z that lie below the rank.  A_K P2
// R_B^{-1} and Algorithm 7's A_K V Sigma^{-1} are both orthonormal bases of
// range(A_K), so the row norms are the same.  The Cholesky runs with
// zeta = 0: B_K's rows and columns past the rank are exact zeros, where it
// stops.
lev_status estimate_exact(const lev_matrix* A, const lev_params* p, int variant, void* theta_out, void* ws,
                          hipStream_t stream) {
  const int64_t n = A->n, d = A->d, m = p->m, r_cs = p->r_cs;
  hipStream_t s = stream;
  Carver c(ws);
  SketchBufs sb = carve_sketch(c, A, p);
  RankBufs rb = carve_rank(c, m, d);
  RefineBufs rf;
  const bool refine = p->zeta < kZetaGram;
  if (refine) rf = carve_refine(c, m, d);
  void* state_ws = c.take<char>(state_bytes(d, m, d));
  ExactBufs eb = carve_exact(c, A, p);
  void* Zpack = c.take<char>(lev::pack_z_bytes(variant, d, d));
  StateView sv = carve_state(state_ws, d, m, d);
  int64_t* rank = sv.header + 4;
  int32_t* err = state_err(sv);
  rb.pc.err = err;
  eb.rb2.pc.err = err;
  const lev::SeedDraws dr = lev::derive_draws(p->seed, n, r_cs);
  LEV_HIP(mark_phase(0, s));
  LEV_HIP(lev::launch_fill_zero(sv.header + 5, sizeof(int64_t), s));
  LEV_TRY(enqueue_sketch(A, p, dr, sb, sb.SA, sv.At, nullptr, s));
  LEV_TRY(enqueue_rank(sv.At, m, d, p->zeta, rb, sv.perm, sv.R, rank, s, refine ? &rf : nullptr));
  LEV_HIP(mark_phase(4, s));
  if (A->format == LEV_CSR) {
    LEV_HIP(lev::launch_gram_csr(A->dtype, A->values, A->row_ptr, A->col_idx, n, d, A->nnz, eb.gram_partial,
                                 eb.C64, s));
  } else if (n > 0) {
    LEV_HIP(lev::launch_gram_dense(A->dtype, A->values, n, d, A->ld, lev::gram_dense_splits(n, d),
                                   eb.gram_partial, eb.C64, s));
  } else {
    LEV_HIP(lev::launch_fill_zero(eb.C64, sizeof(double) * (size_t)(d * d), s));
  }
  LEV_HIP(lev::launch_gather_bk(d, sv.perm, rank, eb.C64, eb.rb2.B, s));
  if (d > 256) LEV_HIP(lev::launch_fill_zero(eb.rb2.pc.flags, 64 * sizeof(int32_t), s));
  LEV_HIP(lev::launch_pivchol(eb.rb2.B, d, 0.0, eb.rb2.pc, eb.rank2, eb.rb2.partial, s));
  LEV_HIP(lev::launch_pivchol_finalize(d, eb.rb2.pc, eb.rank2, eb.perm2, eb.R2, s));
  LEV_HIP(lev::launch_compose_perm(d, sv.perm, eb.perm2, eb.permc, s));
  LEV_HIP(lev::launch_identity(d, eb.I, s));
  LEV_HIP(lev::launch_form_z(variant, d, d, eb.R2, eb.rank2, eb.permc, eb.I, sv.Z64, Zpack, err, s));
  LEV_HIP(mark_phase(5, s));
  if (n > 0 && A->format == LEV_CSR) {
    LEV_HIP(lev::launch_rownorm_csr(A->dtype, A->values, A->row_ptr, A->col_idx, n, d, A->nnz, d, Zpack, eb.rank2,
                                    theta_out, s));
  } else if (n > 0) {
    LEV_HIP(lev::launch_rownorm_dense(variant, A->dtype, A->values, n, d, A->ld, d, Zpack, eb.rank2, theta_out, s));
  }
  LEV_HIP(mark_phase(6, s));
  return LEV_OK;
}

lev_status estimate_qless(const lev_matrix* A, const lev_params* p, int variant, void* theta_out, void* ws,
                          hipStream_t s) {
  const int64_t n = A->n, d = A->d;
  Carver c(ws);
  QlessBufs b = carve_qless(c, A, p);
  const lev::QlessInput in{A->dtype, A->values, A->format == LEV_CSR ? A->row_ptr : nullptr, A->col_idx, n, d,
                           A->ld, A->nnz};
  LEV_HIP(mark_phase(0, s));
  LEV_HIP(lev::launch_fill_zero(b.err, sizeof(int32_t), s));
  LEV_HIP(mark_phase(1, s));
  LEV_HIP(mark_phase(2, s));
  LEV_HIP(mark_phase(3, s));
  LEV_HIP(lev::launch_qless_qr(in, qless_steps(A, p), p->zeta, b.qws, b.perm, b.R, b.rank, s));
  LEV_HIP(mark_phase(4, s));
  LEV_HIP(lev::launch_identity(d, b.I, s));
  LEV_HIP(lev::launch_form_z(variant, d, d, b.R, b.rank, b.perm, b.I, b.Z64, b.Zpack, b.err, s));
  LEV_HIP(mark_phase(5, s));
  if (n > 0 && A->format == LEV_CSR) {
    LEV_HIP(lev::launch_rownorm_csr(A->dtype, A->values, A->row_ptr, A->col_idx, n, d, A->nnz, d, b.Zpack, b.rank,
                                    theta_out, s));
  } else if (n > 0) {
    LEV_HIP(lev::launch_rownorm_dense(variant, A->dtype, A->values, n, d, A->ld, d, b.Zpack, b.rank, theta_out, s));
  }
  LEV_HIP(mark_phase(6, s));
  return LEV_OK;
}

}  // namespace

extern "C" {

lev_status lev_estimate(const lev_matrix* A, const lev_params* p, void* theta_out, void* state_out, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  LEV_TRY(check_matrix(A));
  LEV_TRY(check_params(A, p));
  if (theta_out == nullptr && A->n > 0) return fail(LEV_ERR_ARG, "theta_out is null");
  const size_t need = lev_workspace_size(A, p, LEV_WS_ESTIMATE);
  LEV_TRY(check_ws(ws, ws_bytes, need));
  if (state_out != nullptr && (reinterpret_cast<uintptr_t>(state_out) & (kAlign - 1)) != 0)
    return fail(LEV_ERR_ARG, "state_out must be 256-byte aligned");
  if (state_out != nullptr && p->mode != LEV_MODE_JL)
    return fail(LEV_ERR_NOT_SUPPORTED, "only the JL estimate (LEV_MODE_JL) has a backward state");

  const int64_t n = A->n, d = A->d, m = p->m, r_cs = p->r_cs;
  const int variant = az_variant(A->format, A->dtype, p->az_precision);
  if (p->mode == LEV_MODE_EXACT) return estimate_exact(A, p, variant, theta_out, ws, stream);
  if (p->mode == LEV_MODE_QLESS) return estimate_qless(A, p, variant, theta_out, ws, stream);
  // JL: Z = R11^{-1} G_k (k columns, all live).  No JL step: Z = R11^{-1}
  // [I_r 0] (d columns, the first r live).
  const bool jl = p->mode == LEV_MODE_JL;
  const int64_t k = pass2_cols(A, p);
  Carver c(ws);
  SketchBufs sb = carve_sketch(c, A, p);
  RankBufs rb = carve_rank(c, m, d);
  RefineBufs rf;
  const bool refine = p->zeta < kZetaGram;
  if (refine) rf = carve_refine(c, m, d);
  void* state_ws = c.take<char>(state_bytes(d, m, k));
  double* Gk = c.take<double>((size_t)(d * k));
  void* Zpack = c.take<char>(lev::pack_z_bytes(variant, d, k));
  StateView sv = carve_state(state_out != nullptr ? state_out : state_ws, d, m, k);
  int64_t* rank = sv.header + 4;
  int32_t* err = state_err(sv);
  rb.pc.err = err;
  const int64_t* live = jl ? nullptr : rank;

  const lev::SeedDraws dr = lev::derive_draws(p->seed, n, r_cs);
  LEV_HIP(mark_phase(0, stream));
  LEV_HIP(lev::launch_fill_zero(sv.header + 5, sizeof(int64_t), stream));
  LEV_TRY(enqueue_sketch(A, p, dr, sb, sb.SA, sv.At, jl ? Gk : nullptr, stream));
  LEV_TRY(enqueue_rank(sv.At, m, d, p->zeta, rb, sv.perm, sv.R, rank, stream, refine ? &rf : nullptr));
  LEV_HIP(mark_phase(4, stream));
  if (!jl) LEV_HIP(lev::launch_identity(d, Gk, stream));
  LEV_HIP(lev::launch_form_z(variant, d, k, sv.R, rank, sv.perm, Gk, sv.Z64, Zpack, err, stream));
  LEV_HIP(mark_phase(5, stream));
  if (n > 0 && A->format == LEV_CSR) {
    LEV_HIP(lev::launch_rownorm_csr(A->dtype, A->values, A->row_ptr, A->col_idx, n, d, A->nnz, k, Zpack, live,
                                    theta_out, stream));
  } else if (n > 0) {
    LEV_HIP(lev::launch_rownorm_dense(variant, A->dtype, A->values, n, d, A->ld, k, Zpack, live, theta_out,
                                      stream));
  }
  LEV_HIP(mark_phase(6, stream));
  if (state_out != nullptr) {
    LEV_HIP(lev::launch_store_i64x4(sv.header, kStateMagic, d, m, k, stream));
  }
  return LEV_OK;
}

lev_status lev_estimate_backward(const lev_matrix* A, const lev_params* p, const void* state, const void* w,
                                 void* gradA_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  LEV_TRY(check_matrix(A));
  LEV_TRY(check_params(A, p));
  LEV_TRY(check_backward_input(A, p));
  if (state == nullptr) return fail(LEV_ERR_ARG, "state is null");
  if ((reinterpret_cast<uintptr_t>(state) & (kAlign - 1)) != 0)
    return fail(LEV_ERR_ARG, "state must be 256-byte aligned");
  if (A->n > 0 && (w == nullptr || gradA_out == nullptr)) return fail(LEV_ERR_ARG, "w or gradA_out is null");
  const size_t need = lev_workspace_size(A, p, LEV_WS_BACKWARD);
  LEV_TRY(check_ws(ws, ws_bytes, need));

  const int64_t n = A->n, d = A->d, m = p->m, k = p->k, r_cs = p->r_cs;
  const int dt = A->dtype == LEV_F64 ? 0 : 1;
  Carver c(ws);
  BwdBufs b = carve_bwd(c, A, p);
  const StateView sv = carve_state(const_cast<void*>(state), d, m, k);
  const int64_t* rank = sv.header + 4;
  const lev::SeedDraws dr = lev::derive_draws(p->seed, n, r_cs);
  hipStream_t s = stream;

  // Z_full in the gradient's type (rows by column id, zero off K)
  LEV_HIP(lev::launch_pack_z(dt == 0 ? 6 : 5, d, k, sv.perm, rank, sv.Z64, b.Zpack, s));
  // C = A^T diag(w) A Z_full
  if (n > 0) {
    LEV_HIP(lev::launch_bwd_gram(dt, A->values, n, d, A->ld, k, w, b.Zpack, b.partials, b.groups, b.C64, s));
  } else {
    LEV_HIP(lev::launch_fill_zero(b.C64, sizeof(double) * (size_t)(d * k), s));
  }
  // The FP64 core, at d x d with zeros past the rank (the rank stays on the
  // device): Zbar = 2 C[K]; Rbar = -triu(R11^{-T} Zbar Z^T);
  // N = R11^{-1} copyltu(R11 Rbar^T) R11^{-T}; Abar~_K = A~_K N; H = G^T Abar~_K.
  double *I = b.sq[0], *Rinv = b.sq[1], *T1 = b.sq[2], *X = b.sq[3], *Msym = b.sq[4];
  LEV_HIP(lev::launch_gather_zbar(d, k, sv.perm, rank, b.C64, b.Zbar, s));
  LEV_TRY(gemm(d, d, k, b.Zbar, k, 1, sv.Z64, 1, k, T1, b.gemm_partial, s));          // Zbar Z^T
  LEV_HIP(lev::launch_identity(d, I, s));
  LEV_HIP(lev::launch_trsm_z(d, d, sv.R, rank, I, Rinv, state_err(sv), s));           // R11^{-1}
  LEV_TRY(gemm(d, d, d, Rinv, 1, d, T1, d, 1, X, b.gemm_partial, s));                 // R11^{-T} T1
  LEV_HIP(lev::launch_neg_triu(d, X, s));                                              // Rbar
  double* M1 = I;
  LEV_TRY(gemm(d, d, d, sv.R, d, 1, X, 1, d, M1, b.gemm_partial, s));                 // R11 Rbar^T
  LEV_HIP(lev::launch_copyltu(d, M1, Msym, s));
  double* N1 = T1;
  LEV_TRY(gemm(d, d, d, Rinv, d, 1, Msym, d, 1, N1, b.gemm_partial, s));              // R11^{-1} Msym
  double* N = X;
  LEV_TRY(gemm(d, d, d, N1, d, 1, Rinv, 1, d, N, b.gemm_partial, s));                 // ... R11^{-T}
  LEV_HIP(lev::launch_gather_cols(m, d, sv.perm, rank, sv.At, b.AtK, s));
  LEV_TRY(gemm(m, d, d, b.AtK, d, 1, N, d, 1, b.Abar_t, b.gemm_partial, s));          // A~_K N
  LEV_HIP(lev::launch_gaussian(dr.key_m, m, r_cs, 1.0 / std::sqrt((double)m), b.Gm, s));
  LEV_TRY(gemm(r_cs, d, m, b.Gm, 1, r_cs, b.Abar_t, d, 1, b.H, b.gemm_partial, s));   // G^T Abar~_K
  LEV_HIP(lev::launch_scatter_h(dt, r_cs, d, sv.perm, rank, b.H, b.Hf, s));
  // Abar = 2 diag(w) A Z_full Z_full^T + S^T H_full
  LEV_HIP(lev::launch_bwd_grad(dt, A->values, n, d, A->ld, k, w, b.Zpack, b.Hf, dr.hash, gradA_out, A->ld, s));
  return LEV_OK;
}

}  // extern "C"

namespace {

// Algorithm 11's buffers: the sketch, the rank-revealing step and its
// outputs, and the preconditioner's scratch.
struct PrecondBufs {
  SketchBufs sb;
  RankBufs rb;
  RefineBufs rf;
  double* At;
  double* R;
  int32_t* perm;
  int64_t* rank;
  int32_t* err;
  double* work;
};

PrecondBufs carve_precond(Carver& c, const lev_matrix* A, const lev_params* p) {
  const int64_t d = A->d, m = p->m;
  PrecondBufs b;
  b.sb = carve_sketch(c, A, p);
  b.rb = carve_rank(c, m, d);
  if (p->zeta < kZetaGram) b.rf = carve_refine(c, m, d);
  b.At = c.take<double>((size_t)(m * d));
  b.R = c.take<double>((size_t)(d * d));
  b.perm = c.take<int32_t>((size_t)d);
  b.rank = c.take<int64_t>(1);
  b.err = c.take<int32_t>(1);
  b.work = c.take<double>((size_t)(2 * d * d + d));
  return b;
}

}  // namespace

extern "C" {

size_t lev_precondition_workspace_size(const lev_matrix* A, const lev_params* p) {
  if (check_matrix(A) != LEV_OK || check_params(A, p) != LEV_OK) return 0;
  Carver c(nullptr);
  carve_precond(c, A, p);
  return c.used;
}

lev_status lev_precondition(const lev_matrix* A, const lev_params* p, int method, double* N_out, int64_t* k_out,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  LEV_TRY(check_matrix(A));
  LEV_TRY(check_params(A, p));
  if (method != LEV_PRECOND_QR && method != LEV_PRECOND_SVD)
    return fail(LEV_ERR_ARG, "method must be LEV_PRECOND_QR or LEV_PRECOND_SVD");
  if (method == LEV_PRECOND_SVD && A->d > 128)
    return fail(LEV_ERR_NOT_SUPPORTED, "the SVD preconditioner takes d <= 128 (d = %lld)", (long long)A->d);
  if (N_out == nullptr || k_out == nullptr) return fail(LEV_ERR_ARG, "N_out or k_out is null");
  LEV_TRY(check_ws(ws, ws_bytes, lev_precondition_workspace_size(A, p)));
  const int64_t d = A->d, m = p->m;
  Carver c(ws);
  PrecondBufs b = carve_precond(c, A, p);
  b.rb.pc.err = b.err;
  const lev::SeedDraws dr = lev::derive_draws(p->seed, A->n, p->r_cs);
  const bool refine = p->zeta < kZetaGram;
  LEV_HIP(lev::launch_fill_zero(b.err, sizeof(int32_t), stream));
  LEV_TRY(enqueue_sketch(A, p, dr, b.sb, b.sb.SA, b.At, nullptr, stream));
  LEV_TRY(enqueue_rank(b.At, m, d, p->zeta, b.rb, b.perm, b.R, b.rank, stream, refine ? &b.rf : nullptr));
  LEV_HIP(lev::launch_precondition(method, d, b.R, b.rank, b.perm, p->zeta, b.work, N_out, k_out, b.err, stream));
  LEV_HIP(lev::launch_flag_error(b.err, k_out, stream));
  return LEV_OK;
}

size_t lev_lsqr_workspace_size(const lev_matrix* A) {
  if (check_matrix(A) != LEV_OK || A->format != LEV_DENSE_ROWMAJOR) return 0;
  return align_up(sizeof(double) * lev::lsqr_ws_doubles(A->n, A->d));
}

lev_status lev_lsqr(const lev_matrix* A, const double* N, const double* b, int64_t iters, double* x_out,
                    double* resid_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  LEV_TRY(check_matrix(A));
  if (A->format != LEV_DENSE_ROWMAJOR) return fail(LEV_ERR_NOT_SUPPORTED, "LSQR takes dense A only");
  if (iters < 0) return fail(LEV_ERR_ARG, "iters = %lld < 0", (long long)iters);
  if (N == nullptr || x_out == nullptr || (A->n > 0 && b == nullptr)) return fail(LEV_ERR_ARG, "null pointer argument");
  LEV_TRY(check_ws(ws, ws_bytes, lev_lsqr_workspace_size(A)));
  LEV_HIP(lev::launch_lsqr(A->dtype, A->values, A->n, A->d, A->ld, N, b, iters, x_out, resid_out,
                           static_cast<double*>(ws), stream));
  return LEV_OK;
}

size_t lev_noalloc_max_bytes(void) { return kScratchBytes; }

lev_status lev_estimate_noalloc(const lev_matrix* A, const lev_params* p, void* theta_out, hipStream_t stream) {
  // every check that needs no device comes first: a request beyond the
  // scratch array is refused before the device is touched
  LEV_TRY(check_matrix(A));
  LEV_TRY(check_params(A, p));
  const size_t need = lev_workspace_size(A, p, LEV_WS_ESTIMATE);
  if (need > kScratchBytes)
    return fail(LEV_ERR_WORKSPACE,
                "lev_estimate_noalloc: this problem needs %zu bytes of workspace, more than the %zu-byte "
                "static scratch; use lev_estimate with a caller-provided workspace",
                need, kScratchBytes);
  int dev = 0;
  LEV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LEV_ERR_NOT_SUPPORTED, "device index %d out of range", dev);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || ptr == nullptr)
        return fail(LEV_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      g_scratch_ptr[dev] = ptr;
    }
    ws = g_scratch_ptr[dev];
  }
  return lev_estimate(A, p, theta_out, nullptr, ws, kScratchBytes, stream);
}

lev_status lev_debug_hash(uint64_t seed, int64_t n, int64_t r_cs, int64_t* h_out, int8_t* s_out,
                          hipStream_t stream) {
  if (n < 0 || n > kMaxRows || r_cs < 1 || r_cs > kMaxRows) return fail(LEV_ERR_SHAPE, "bad n or r_cs");
  if (n > 0 && (h_out == nullptr || s_out == nullptr)) return fail(LEV_ERR_ARG, "null output");
  const lev::SeedDraws dr = lev::derive_draws(seed, n, r_cs);
  LEV_HIP(lev::launch_hash_rows(dr.hash, h_out, s_out, stream));
  return LEV_OK;
}

lev_status lev_hash_params(uint64_t seed, int64_t n, int64_t r_cs, uint64_t* out) {
  if (n < 0 || n > kMaxRows || r_cs < 1 || r_cs > kMaxRows) return fail(LEV_ERR_SHAPE, "bad n or r_cs");
  if (out == nullptr) return fail(LEV_ERR_ARG, "out is null");
  const lev::SeedDraws dr = lev::derive_draws(seed, n, r_cs);
  const lev::HashParams& h = dr.hash;
  const uint64_t v[7] = {h.P, h.a, h.c, h.c0, h.c1, h.c2, h.c3};
  for (int i = 0; i < 7; ++i) out[i] = v[i];
  return LEV_OK;
}

lev_status lev_debug_buckets(uint64_t seed, int64_t n, int64_t r_cs, int64_t* bucket_off, int32_t* bucket_rows,
                             hipStream_t stream) {
  if (n < 0 || n > kMaxRows || r_cs < 1 || r_cs > kMaxRows) return fail(LEV_ERR_SHAPE, "bad n or r_cs");
  if (bucket_off == nullptr || (n > 0 && bucket_rows == nullptr)) return fail(LEV_ERR_ARG, "null output");
  const lev::SeedDraws dr = lev::derive_draws(seed, n, r_cs);
  LEV_HIP(lev::launch_bucket_lists(dr.hash, bucket_off, bucket_rows, stream));
  return LEV_OK;
}

lev_status lev_debug_gaussian(uint64_t seed, int which, int64_t rows, int64_t cols, double* out,
                              hipStream_t stream) {
  if (rows < 1 || cols < 1) return fail(LEV_ERR_SHAPE, "rows and cols must be >= 1");
  if (out == nullptr) return fail(LEV_ERR_ARG, "out is null");
  if (which != 0 && which != 1) return fail(LEV_ERR_ARG, "which must be 0 or 1");
  const lev::SeedDraws dr = lev::derive_draws(seed, 2, 1);
  const double scale = 1.0 / std::sqrt((double)(which == 0 ? rows : cols));
  LEV_HIP(lev::launch_gaussian(which == 0 ? dr.key_m : dr.key_k, rows, cols, scale, out, stream));
  return LEV_OK;
}

lev_status lev_debug_stream_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t stream) {
  if (buf == nullptr || sink == nullptr) return fail(LEV_ERR_ARG, "buf and sink must not be null");
  if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0) return fail(LEV_ERR_ARG, "buf must be 16-byte aligned");
  if (bytes <= 0 || bytes % 16 != 0) return fail(LEV_ERR_ARG, "bytes must be a positive multiple of 16");
  LEV_HIP(lev::launch_stream_read(buf, bytes, sink, stream));
  return LEV_OK;
}

}  // extern "C"
