// Internal interface between the C API (lev_api.cpp) and the kernels.
// Not installed; nothing outside csrc/ includes it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lev {

// Parameters of the CountSketch S, expanded from the user seed on the host.
// Bucket hash: h(i) = ((a*i + c) mod P) mod r_cs with P the smallest prime
// >= max(n, 2) (P < 2^32 since n < 2^31).  Pass 1 walks bucket b by
// inverting the permutation x = (a*i + c) mod P: the rows of bucket b are
// i = ainv * (x - c) mod P for x = b, b + r_cs, b + 2 r_cs, ... < P, kept
// when i < n, i.e. the arithmetic progression i_t = i_0 + t*delta (mod P)
// with delta = ainv * r_cs mod P.
// Sign: s(i) = +1 if (c3 i^3 + c2 i^2 + c1 i + c0) mod (2^61 - 1) is even.
struct HashParams {
  uint64_t P, a, c, ainv, delta;
  uint64_t pbar;  // floor((2^64 - 1) / P): Barrett reduction mod P (P < 2^32)
  uint64_t c0, c1, c2, c3;
  int64_t n, r_cs;
};

struct PhiloxKey {
  uint32_t k0, k1;
};

struct SeedDraws {
  HashParams hash;
  PhiloxKey key_m;  // Gaussian transform G_m
  PhiloxKey key_k;  // JL Gaussian G_k
  uint64_t key_d;   // SRHT signs D
  uint64_t key_p;   // SRHT coordinate sample P
};

// Host-side expansion of a seed (SplitMix64 words w0..w9).
SeedDraws derive_draws(uint64_t seed, int64_t n, int64_t r_cs);

// ---- launch wrappers (all enqueue on `s`, return hipError_t of the launch) ----

// h(i), s(i) for all rows (debug/inspection).
hipError_t launch_hash_rows(const HashParams& hp, int64_t* h_out, int8_t* s_out, hipStream_t s);
// bucket_off[r_cs+1], bucket_rows[n] in pass-1 order (debug/inspection).
hipError_t launch_bucket_lists(const HashParams& hp, int64_t* off, int32_t* rows, hipStream_t s);

// Up to two Gaussian matrices drawn by pass 1 on the side (each the draws
// of launch_gaussian: element e = pair e / 2 of its Philox stream, times its
// scale): the bucket workgroups each take an equal share of the pairs of
// both, so the FP64 transcendentals run while the CUs stream A.  A matrix
// with out == nullptr is not drawn.
struct GaussMatrix {
  PhiloxKey key;
  int64_t total;  // elements
  double scale;
  double* out;
  // instead of out (FP64): the values rounded to FP32 and split exactly
  // into three BF16 parts, part p of element e at BF16 index
  // p * 2 * ceil(total / 2) + e (the operand of launch_xgemm)
  uint32_t* parts3 = nullptr;
};
struct GaussDraw {
  GaussMatrix m[2];
};

// Pass 1, dense: SA (r_cs x d, ld = d) = S A, plus the draw g.  The sums
// are taken in FP64; sa_f32: SA is stored as float (rounded once at the
// store), otherwise as double.  dtype: 0 = f64, 1 = f32, 2 = bf16.
hipError_t launch_countsketch_dense(int dtype, const void* A, int64_t n, int64_t d, int64_t ld,
                                    const HashParams& hp, void* SA, bool sa_f32, const GaussDraw& g,
                                    hipStream_t s);
// Pass 1, CSR (row_ptr int64[n+1], col_idx int32[nnz], vals[nnz]), plus the
// draw g.  Row extents are clamped to [0, nnz] and to d entries, column ids
// >= d skipped.
hipError_t launch_countsketch_csr(int dtype, const void* vals, const int64_t* row_ptr,
                                  const int32_t* col_idx, int64_t n, int64_t d, int64_t nnz,
                                  const HashParams& hp, double* SA, const GaussDraw& g, hipStream_t s);

// rows x cols FP64 Gaussian matrix, Philox4x32-10 + Box-Muller, times scale.
hipError_t launch_gaussian(PhiloxKey key, int64_t rows, int64_t cols, double scale, double* out,
                           hipStream_t s);

// The SRHT F = P H D / sqrt(t) (srht.hip) applied to X = S A (r x d FP64,
// r a power of two, overwritten by H D X): At (t x d) = F X.  inv: int32[r]
// scratch (the sampled coordinates).
hipError_t launch_srht(uint64_t key_d, uint64_t key_p, int64_t r, int64_t d, int64_t t, double* X, int32_t* inv,
                       double* At, hipStream_t s);

// FP64 GEMM on MFMA: C = alpha * op(A) op(B) + beta * C with arbitrary
// element strides: op(A)(i,k) = A[i*sai + k*sak], op(B)(k,j) = B[k*sbk + j*sbj],
// C(i,j) = C[i*ldc + j].  If `skip` is non-null and *skip != 0 on the device,
// the kernel does nothing.  `partial` (splits * M * N doubles) is used when
// splits > 1 (split-K, reduced in fixed order).
hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sai,
                        int64_t sak, const double* B, int64_t sbk, int64_t sbj, double beta,
                        double* C, int64_t ldc, int splits, double* partial, const int32_t* skip,
                        hipStream_t s);
size_t dgemm_partial_elems(int64_t M, int64_t N, int splits);
int dgemm_choose_splits(int64_t M, int64_t N, int64_t K);

// Pivoted Cholesky of the d x d Gram B (overwritten with Schur complements).
struct PivCholState {
  double* diag = nullptr;     // d
  double* Rrows = nullptr;    // d x d: row J = row J of R in original column order
  int32_t* piv = nullptr;     // d: pivot at position J
  int32_t* flags = nullptr;   // [0] = done, [1] = pivots so far, [2..] scratch
  double* r00 = nullptr;      // 1
  int32_t* err = nullptr;     // optional: bit kErrPivotWait is set when a bounded wait ran out
};

// Bits of the device error word (state header, slot 5).  A bounded wait
// inside a kernel that runs out sets its bit and ends that kernel's work
// early, so the results of the call are then meaningless; the word is
// cleared at the start of every estimate.
constexpr int32_t kErrPivotWait = 1;
constexpr int32_t kErrSolveWait = 2;
// fixed != 0: no pivoting (step J takes column J), i.e. the plain Cholesky
// of B, stopping at the first non-positive diagonal.  ref_r00 (device, may
// be null): the R_00 the cutoff zeta * R_00 refers to, instead of the first
// pivot's own.
hipError_t launch_pivchol(double* B, int64_t d, double zeta, const PivCholState& st, int64_t* rank_out,
                          double* gemm_partial, hipStream_t s, int fixed = 0, const double* ref_r00 = nullptr);
// Writes perm (int32[d], unpivoted columns ascending after the rank) and
// R_out (d x d, pivoted order, zero below the diagonal and below the rank).
hipError_t launch_pivchol_finalize(int64_t d, const PivCholState& st, const int64_t* rank,
                                   int32_t* perm_out, double* R_out, hipStream_t s);

// Z = R11^{-1} G_k[0:r, 0:k] in FP64 (R pivoted d x d, ld = d), r read from
// the device.  Z64 is d x k (rows >= r zeroed).  For d > 256 the solve runs
// over diagonal blocks of 256 and G's rows above the last block are
// overwritten (they carry the updated right-hand side).
// err (may be null): bit kErrSolveWait is set if a bounded wait runs out.
hipError_t launch_trsm_z(int64_t d, int64_t k, const double* R, const int64_t* rank, double* G, double* Z64,
                         int32_t* err, hipStream_t s);

// Prepares the operand of pass 2: Z_full (d x k, rows indexed by original
// column, zero off K) converted to the pass-2 compute type and laid out for
// the MFMA B-operand; see rownorm.hip for the layouts.  For k > 64 the
// operand is a sequence of column tiles of 64 (the last one ragged), each
// packed as if it were the whole of a k <= 64 operand: tile t starts at
// byte pack_z_tile_offset(variant, d, k, t), and pass 2 makes one pass over
// A per tile (ColTile below).
// variant: 0 = FP64, 1 = FP32, 2 = BF16, 3 = BF16 hi/lo, 4 = BF16x3 (FP32 A),
// 5 = FP32 row-major d x 64 (CSR pass 2), 6 = FP64 row-major d x 64 (CSR).
// pack_z_bytes: workspace needed (operand + an inverse permutation);
// pack_z_operand_bytes: the operand alone (what pass 2 reads).
hipError_t launch_pack_z(int variant, int64_t d, int64_t k, const int32_t* perm, const int64_t* rank,
                         const double* Z64, void* Zpack, hipStream_t s);
size_t pack_z_bytes(int variant, int64_t d, int64_t k);
// trsm + pack in one launch where it fits (d <= 256, k <= 64), else the
// launches above (Gk overwritten as there).  Zpack as for launch_pack_z.
hipError_t launch_form_z(int variant, int64_t d, int64_t k, const double* R, const int64_t* rank,
                         const int32_t* perm, double* Gk, double* Z64, void* Zpack, int32_t* err,
                         hipStream_t s);
size_t pack_z_operand_bytes(int variant, int64_t d, int64_t k);
constexpr int64_t kZTile = 64;
inline int64_t z_tiles(int64_t k) { return (k + kZTile - 1) / kZTile; }
size_t pack_z_tile_offset(int variant, int64_t d, int64_t k, int64_t t);

// One column tile of pass 2 (k > 64 runs one pass per tile of 64 columns).
// live (device, may be null): the number of leading columns of Z that can
// be nonzero; the pass returns at once when *live <= c0 (its tile is all
// zero).  acc != 0: theta += the tile's squares instead of theta = them.
struct ColTile {
  const int64_t* live = nullptr;
  int64_t c0 = 0;
  int32_t acc = 0;
};
__device__ __forceinline__ bool col_tile_dead(const ColTile& ct) { return ct.live != nullptr && *ct.live <= ct.c0; }

// Pass 2, dense: theta[i] = || A[i, :] Z_full ||^2.
// variant as above; dtype = storage type of A (0 f64, 1 f32, 2 bf16).
// live (device, may be null): columns >= *live of Z are known to be zero,
// so their tiles are skipped (k > 64 only).
hipError_t launch_rownorm_dense(int variant, int dtype, const void* A, int64_t n, int64_t d, int64_t ld,
                                int64_t k, const void* Zpack, const int64_t* live, void* theta,
                                hipStream_t s);
// Pass 2 for BF16 storage (rownorm_bf16.hip): one tile (k <= 64) of Z_full
// packed as variant 2 (parts = 1), 3 (parts = 2) or 4 (parts = 3); theta FP32.
hipError_t launch_rownorm_bf16(int parts, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k,
                               const void* Zpack, void* theta, const ColTile& ct, hipStream_t s);
// Pass 2, CSR: theta[i] = || A[i, :] Z_full ||^2 with Z_full packed by
// launch_pack_z as variant 5 (FP32, for F32/BF16 values) or 6 (FP64, for
// F64 values): per tile, d rows of 64 elements (columns >= k zero).  theta
// is FP64 for F64 values, else FP32.  live as for launch_rownorm_dense.
hipError_t launch_rownorm_csr(int dtype, const void* vals, const int64_t* row_ptr, const int32_t* col_idx,
                              int64_t n, int64_t d, int64_t nnz, int64_t k, const void* Zpack,
                              const int64_t* live, void* theta, hipStream_t s);

// Algorithm 6 (qless.hip): Q-less column-pivoted QR of A itself, kmax
// steps at most, stopping before r_jj <= zeta r_00.  Writes perm (int32[d]:
// the pivots, then the other columns ascending), R_out (d x d, pivoted
// order, zero past the rank) and rank (device).  ws: qless_ws_doubles
// doubles.  row_ptr == nullptr: dense row-major A (ld), else CSR.
struct QlessInput {
  int dtype;  // 0 f64, 1 f32, 2 bf16
  const void* values;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  int64_t n, d, ld, nnz;
};
int qless_groups(int64_t n, bool csr);
size_t qless_ws_doubles(int64_t n, int64_t d, int64_t kmax, bool csr);
hipError_t launch_qless_qr(const QlessInput& in, int64_t kmax, double zeta, double* ws, int32_t* perm_out,
                           double* R_out, int64_t* rank_out, hipStream_t st);

// Section 6 (precond.hip).  method 0: N = P R11^{-1}; 1: N = P V_R
// Sigma^{-1} from a one-sided Jacobi SVD of R (d <= 128), keeping sigma_j >
// zeta sigma_1.  N is d x d row-major (columns past k zero); work: 2 d^2 + d
// doubles; k_out on the device.
hipError_t launch_precondition(int method, int64_t d, const double* R, const int64_t* rank, const int32_t* perm,
                               double zeta, double* work, double* N, int64_t* k_out, int32_t* err, hipStream_t s);
hipError_t launch_flag_error(const int32_t* err, int64_t* k_out, hipStream_t s);
// LSQR on A N (dense A of dtype 0/1/2) from y = 0, iters steps, x = N y;
// hist (may be null): the residual-norm estimate after each step.
int lsqr_groups(int64_t n);
size_t lsqr_ws_doubles(int64_t n, int64_t d);
hipError_t launch_lsqr(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, const double* N, const double* b,
                       int64_t iters, double* x, double* hist, double* ws, hipStream_t s);

// A streaming read of `bytes` (a multiple of 16) at buf: the measured read
// ceiling (probe.hip); sink holds stream_read_sink_len() checksums.
int64_t stream_read_sink_len();
hipError_t launch_stream_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t s);

// B (d x d, FP64) = A^T A for dense A (dtype 0 f64, 1 f32, 2 bf16) on the
// FP64 matrix cores: the products of FP32 and BF16 elements are exact in
// FP64.  partial: dgemm_partial_elems(d, d, splits) doubles.
hipError_t launch_gram_dense(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int splits,
                             double* partial, double* B, hipStream_t s);
int gram_dense_splits(int64_t n, int64_t d);
// Splits (>= 2) for the sketch's Gram through launch_gram_dense (FP64 A~, m rows).
int gram_sketch_splits(int64_t m, int64_t d);
// B (d x d, FP64) = A^T A for CSR A in sum_i nnz_i^2 work (gram_csr.hip).
size_t gram_csr_partial_elems(int64_t n, int64_t d);
hipError_t launch_gram_csr(int dtype, const void* vals, const int64_t* row_ptr, const int32_t* col_idx,
                           int64_t n, int64_t d, int64_t nnz, double* partial, double* B, hipStream_t s);

// ---- backward (adjoint of w^T theta~ at a fixed sketch) ----------------------
// dtype 0 = FP64, 1 = FP32 (A, w, Z_full, H_full and the gradient share it).
// Z_full is the variant-5/6 packing (d rows of 64).
int bwd_groups(int dtype, int64_t n, int64_t d, int64_t k);
size_t bwd_elem_size(int dtype);
// C64 (d x k, FP64) = A^T diag(w) A Z_full; partials: groups x d x 64 elements.
hipError_t launch_bwd_gram(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w,
                           const void* Zfull, void* partials, int groups, double* C64, hipStream_t s);
// G (n x ldg) = 2 diag(w) A Z_full Z_full^T + S^T H_full (H_full r_cs x d).
hipError_t launch_bwd_grad(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w,
                           const void* Zfull, const void* Hfull, const HashParams& hp, void* G, int64_t ldg,
                           hipStream_t s);
hipError_t launch_gather_zbar(int64_t d, int64_t k, const int32_t* perm, const int64_t* rank, const double* C64,
                              double* Zbar, hipStream_t s);
hipError_t launch_neg_triu(int64_t d, double* X, hipStream_t s);
hipError_t launch_copyltu(int64_t d, const double* M, double* out, hipStream_t s);
hipError_t launch_identity(int64_t d, double* I, hipStream_t s);
hipError_t launch_gather_cols(int64_t m, int64_t d, const int32_t* perm, const int64_t* rank, const double* At,
                              double* AtK, hipStream_t s);
hipError_t launch_scatter_h(int dtype, int64_t rows, int64_t d, const int32_t* perm, const int64_t* rank,
                            const double* H, void* Hf, hipStream_t s);

// ---- refined rank-revealing factorisation (rrqr.hip) --------------------------
// X1 = A~[:, perm[0..r)] with the other columns zero, X2 = the rest (may be
// null), both m x d in perm order.
hipError_t launch_gather_split(int64_t m, int64_t d, const int32_t* perm, const int64_t* rank, const double* At,
                               double* X1, double* X2, hipStream_t s);
// dst += a + b
hipError_t launch_add2(int64_t n, double* dst, const double* a, const double* b, hipStream_t s);
// Final perm, R and rank from stage 1 (perm1, r1, rows Rtop) and stage 2
// (perm2 as positions of perm1, r2, rows Rbot); see rrqr.hip.
hipError_t launch_rrqr_assemble(int64_t d, const int32_t* perm1, const int64_t* rank1, const int32_t* perm2,
                                const int64_t* rank2, const double* Rtop, const double* Rbot, int32_t* perm_out,
                                double* R_out, int64_t* rank_out, hipStream_t s);
// *flag = (*rank == d)
hipError_t launch_full_rank_flag(int64_t d, const int64_t* rank, int32_t* flag, hipStream_t s);

// ---- the Gaussian transform in FP32-level arithmetic (xgemm.hip) -------------
// out (3 parts of N x K BF16, rows contiguous in k) = the three-part split
// of SA^T (SA K x N row-major, float when sa_f32, else double, split from
// its FP32 value either way); K even.
hipError_t launch_split_t3(int64_t K, int64_t N, const void* SA, bool sa_f32, void* out, hipStream_t s);
// C (M x N FP64, row stride ldc) = A B^T from three-part operands: Ap 3
// parts of M x K, Bp 3 parts of N x K (BF16, rows of K elements, K a
// multiple of 8), the six products above 2^-24 on BF16 MFMAs, FP32 within a
// 32-wide K step, FP64 beyond; partial: splits x M x N FP64 when splits > 1.
hipError_t launch_xgemm(int64_t M, int64_t N, int64_t K, const void* Ap, const void* Bp, double* C, int64_t ldc,
                        int splits, double* partial, hipStream_t s);
int xgemm_choose_splits(int64_t M, int64_t N, int64_t K);
size_t xgemm_partial_elems(int64_t M, int64_t N, int splits);
// BF16 elements of one part of a three-part split of rows x K (K rounded up to even)
size_t split3_elems(int64_t rows, int64_t K);

// dst[0..3] = (a, b, c, e) from a kernel (capture-safe small header write).
hipError_t launch_store_i64x4(int64_t* dst, int64_t a, int64_t b, int64_t c, int64_t e, hipStream_t s);

// Zero-fill helper (a kernel, so it is safe under graph capture).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// LS-HRN-exact (Algorithm 7): B_K = C[K, K] (zeros past the rank) and
// permc[j] = perm[perm2[j]].
hipError_t launch_gather_bk(int64_t d, const int32_t* perm, const int64_t* rank, const double* C, double* B,
                            hipStream_t s);
hipError_t launch_compose_perm(int64_t d, const int32_t* perm, const int32_t* perm2, int32_t* permc, hipStream_t s);

}  // namespace lev
