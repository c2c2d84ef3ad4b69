/*
 * lev.h -- C interface of liblev, an MI355X (gfx950) implementation of the
 * randomized row-leverage-score estimator LS-HRN-approx of Sobczyk &
 * Gallopoulos, "Estimating leverage scores via rank revealing methods and
 * randomization" (Algorithm 10: Algorithm 4 followed by Algorithm 8 on the
 * selected columns).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All matrix/vector pointers are DEVICE pointers (hipMalloc'd or owned by
 *   a framework such as PyTorch) unless a comment says "host".  The caller
 *   owns every buffer; the library never allocates, frees or synchronises.
 *   Work is enqueued on the caller's stream and completes in stream order.
 * - Dense matrices are row-major with a leading dimension `ld` (elements
 *   between consecutive rows, ld >= d).
 * - Scratch memory comes from a caller-provided workspace `ws` of
 *   `ws_bytes` bytes; query the size with lev_workspace_size().  The
 *   workspace must be 256-byte aligned.
 * - Return value: LEV_OK (0) or a negative lev_status.  All argument
 *   validation happens on the host BEFORE anything is enqueued; on error
 *   nothing has been launched and the outputs are untouched.  Faults inside
 *   kernels surface at the caller's next synchronisation.  A readable
 *   message for the most recent error of the calling thread is returned by
 *   lev_last_error().
 * - Random draws (the CountSketch hash and signs, the Gaussian transform
 *   G_m and the JL Gaussian G_k) are all derived from params->seed, so two
 *   calls with the same seed and shapes use the same sketch.  Their exact
 *   definitions (SplitMix64 seed expansion, Carter-Wegman bucket hash over
 *   the smallest prime P >= n, cubic sign polynomial over GF(2^61-1),
 *   Philox4x32-10 + Box-Muller) are documented in the repository's design
 *   notes.
 */
#ifndef LEV_H
#define LEV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lev_status;
enum {
  LEV_OK = 0,
  LEV_ERR_ARG = -1,           /* null pointer, bad enum, bad parameter value */
  LEV_ERR_SHAPE = -2,         /* inconsistent or unsupported sizes */
  LEV_ERR_DTYPE = -3,         /* dtype not supported by this call */
  LEV_ERR_FORMAT = -4,        /* malformed CSR (checked only where stated) */
  LEV_ERR_WORKSPACE = -5,     /* ws too small or misaligned */
  LEV_ERR_HIP = -6,           /* a HIP runtime call failed at launch */
  LEV_ERR_NOT_SUPPORTED = -7  /* valid request the library does not handle */
};

enum { LEV_DENSE_ROWMAJOR = 0, LEV_CSR = 1 };
enum { LEV_F64 = 0, LEV_F32 = 1, LEV_BF16 = 2 };

/* Arithmetic of the pass that forms A_{:,K} Z and its squared row norms
 * (Algorithm 8, last step).  Dense A:
 *  NATIVE: F64 input -> FP64 MFMA; F32 input -> BF16X3; BF16 input -> BF16.
 *  FP32:   FP32 MFMA (16x16x4), any storage type but F64.
 *  BF16:   BF16 MFMA with Z rounded to BF16 (BF16 input only).
 *  BF16X2: BF16 MFMA, Z split into a BF16 high and low part (BF16 input only).
 *  BF16X3: FP32 input: A and Z are each split exactly into three BF16
 *          parts (24 significant bits, like FP32) and the six products above
 *          2^-24 relative run on the BF16 matrix cores: FP32-level accuracy at
 *          a fraction of the FP32 matrix-core time.  BF16 input: A is exact
 *          in BF16, so only Z is split into three parts (three products):
 *          the FP32-level form of the BF16-stored estimator.
 * MFMA accumulators are FP32 (FP64 for F64 input) and are added into FP64
 * accumulators after every contraction chunk of 8-32 columns (BF16 input:
 * every 4 chunks of 32, i.e. runs of 128 products).
 * CSR A (no dense tile for the matrix cores): NATIVE or FP32 -> FP32 vector
 * FMAs (FP64 for F64 values, NATIVE only). */
enum { LEV_AZ_NATIVE = 0, LEV_AZ_FP32 = 1, LEV_AZ_BF16 = 2, LEV_AZ_BF16X2 = 3, LEV_AZ_BF16X3 = 4 };

/* The tall input A (n x d, n >> d).
 *  DENSE_ROWMAJOR: values points at n*ld elements of `dtype`; row_ptr and
 *    col_idx are ignored.  values must be 16-byte aligned and ld*sizeof(elt)
 *    a multiple of 16 bytes (d itself may be anything <= ld).
 *  CSR: row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] =
 *    nnz), col_idx int32[nnz] strictly increasing within each row and < d,
 *    values[nnz] of `dtype`; ld is ignored.  The CSR invariants are the
 *    caller's responsibility: the kernels clamp row extents to [0, nnz] and
 *    skip column ids >= d, so a malformed matrix gives wrong scores but no
 *    access outside the arrays (given a correct nnz). */
typedef struct {
  int32_t format;
  int32_t dtype;
  int64_t n, d, ld, nnz;
  const void* values;
  const int64_t* row_ptr;
  const int32_t* col_idx;
} lev_matrix;

/* Parameters of the estimator.
 *  seed  -- 64-bit seed of all random draws.
 *  r_cs  -- rows of the CountSketch S (Algorithm 3's r).  >= 1.
 *  m     -- rows of the Gaussian transform G (Algorithm 3's m = ceil(gamma d)).
 *           d <= m required.
 *  k     -- columns of the JL Gaussian Pi_2 (Algorithm 8's r_2).  1..4096
 *           (the backward pass takes k <= 64).  Pass 2 makes one pass over
 *           A per 64 columns.  LEV_MODE_QLESS: the step cap; ignored by the
 *           other modes.
 *  zeta  -- rank tolerance: the revealed rank is r = #{ j : R_jj > zeta R_00 }
 *           on the column-pivoted factor of the sketch (the cutoff rule of
 *           Section 7).  Supported: 1e-10 <= zeta < 1 (1e-10 is the FP64
 *           cutoff of the paper's experiments); smaller values give
 *           LEV_ERR_NOT_SUPPORTED, values outside [0, 1) LEV_ERR_ARG.
 *           (lev_sketch ignores zeta.)
 *  az_precision -- LEV_AZ_* above.
 *  mode  -- what lev_estimate returns (LEV_MODE_* below); lev_estimate's
 *           state_out must be NULL unless mode is LEV_MODE_JL.
 *  sketch -- the dense stage after the CountSketch (LEV_SKETCH_* below). */
typedef struct {
  uint64_t seed;
  int64_t r_cs, m, k;
  double zeta;
  int32_t az_precision;
  int32_t mode;
  int32_t sketch;
} lev_params;

/* LEV_SKETCH_GAUSS: A~ = G (S A) with the m x r_cs Gaussian G / sqrt(m)
 *   (Algorithm 3, the CountGauss sketch).
 * LEV_SKETCH_SRHT: A~ = F (S A) with the m x r_cs SRHT F = sqrt(r_cs / m)
 *   P (H / sqrt(r_cs)) D of Section 3.4 (the F S composition of Section 4):
 *   D random signs, H the Walsh-Hadamard matrix, P the first m coordinates
 *   of a keyed permutation of [0, r_cs).  Needs r_cs a power of two and
 *   m <= r_cs (LEV_ERR_ARG / LEV_ERR_SHAPE otherwise); the product costs
 *   r_cs d log2(r_cs) additions instead of 2 m r_cs d flops.  The backward
 *   pass takes LEV_SKETCH_GAUSS only. */
enum { LEV_SKETCH_GAUSS = 0, LEV_SKETCH_SRHT = 1 };

/* LEV_MODE_JL: Algorithm 10 (LS-HRN-approx): theta~_i = ||e_i^T A_K
 *   R11^{-1} Pi_2||^2 with the k-column JL Gaussian Pi_2.
 * LEV_MODE_NOJL: the same estimator without the JL step (Pi_2 = I, i.e.
 *   Algorithm 8 with r_2 = r): theta'_i = ||e_i^T A_K R11^{-1}||^2, the
 *   estimate the JL step approximates; pass 2 runs over ceil(r / 64) column
 *   tiles.
 * LEV_MODE_EXACT: Algorithm 7 (LS-HRN-exact): the same columns K and rank r
 *   from the sketch, then the exact leverage scores of A_K from B = A_K^T
 *   A_K (Algorithm 5's Gram route): one more pass over A for B (dense: FP64
 *   matrix cores, 2 n d^2 flops; CSR: sum_i nnz_i^2 products), the pivoted
 *   Cholesky B_K P2 = R_B^T R_B, and theta~_i = ||e_i^T A_K P2 R_B^{-1}||^2
 *   over ceil(r / 64) column tiles.  The CSR Gram adds its FP64 products
 *   with LDS atomics, so its last bits can differ between runs.
 * LEV_MODE_QLESS: Algorithm 6: exact scores from a Q-less column-pivoted QR
 *   of A itself (no sketch: m, r_cs and sketch are not used): step j
 *   takes the column of largest remaining norm, forms row j of R from the
 *   column inner products A^T a_p (one pass over A per step) and downdates
 *   the norms; it stops before R_jj <= zeta R_00 or after k steps (k is the
 *   step cap here, any k >= 1, at most d steps run).  Then theta_i =
 *   ||e_i^T A P_k R_k^{-1}||^2.  The cutoff is read off downdated norms, so
 *   zeta >= 1e-5 (LEV_ERR_NOT_SUPPORTED below).  Meant for small ranks. */
enum { LEV_MODE_JL = 0, LEV_MODE_EXACT = 1, LEV_MODE_NOJL = 2, LEV_MODE_QLESS = 3 };

/* Workspace bytes needed by lev_sketch (which = LEV_WS_SKETCH),
 * lev_estimate (LEV_WS_ESTIMATE) or lev_estimate_backward (LEV_WS_BACKWARD)
 * for this A and p; lev_rank_workspace_size gives lev_rank_estimate's.
 * Both return 0 when the arguments are invalid. */
enum { LEV_WS_SKETCH = 0, LEV_WS_ESTIMATE = 2, LEV_WS_BACKWARD = 3 };
size_t lev_workspace_size(const lev_matrix* A, const lev_params* p, int which);
size_t lev_rank_workspace_size(int64_t m, int64_t d);

/* Bytes of the state blob written by lev_estimate for lev_estimate_backward. */
size_t lev_state_size(int64_t d, int64_t m, int64_t k);

/* Algorithm 3 (CountGaussSketch): A~ = G (S A), with S the r_cs x n
 * CountSketch (S[h(i), i] = s(i), Section 3.4) and G = G_m / sqrt(m) an
 * m x r_cs Gaussian embedding (Section 3.4, Gaussian embeddings).
 *  At_out     -- m x d, FP64, row-major (ld = d).
 *  SA_out     -- optional (NULL to skip): r_cs x d FP64 copy of S A.
 * S A is accumulated in FP64 in a fixed order (deterministic bits).
 * Supported: dense and CSR, F64/F32/BF16 values. */
lev_status lev_sketch(const lev_matrix* A, const lev_params* p, double* At_out,
                      double* SA_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 4, steps 2-3, on an m x d FP64 sketch At (row-major, ld = d):
 * column-pivoted QR of At (Businger-Golub pivoting: the next pivot is the
 * remaining column of largest residual norm; exact ties go to the lowest
 * column index), R sign-normalised to a non-negative diagonal, and the rank
 * r = #{ j : R_jj > zeta R_00 }.  Pivoting stops at r.
 *  perm_out -- int32[d]: perm_out[j] = original column at pivot position j;
 *              entries j >= r list the unselected columns in ascending order.
 *  R_out    -- d x d FP64 row-major; rows j < r hold row j of the pivoted,
 *              upper-triangular factor (R_out[j][t] for t >= j, zeros left of
 *              the diagonal); rows j >= r are zero.
 *  rank_out -- device int64 scalar r.
 * Computed without Householder reflections, from the Gram matrix and
 * Cholesky QR: for zeta >= 1e-5 the pivoted Cholesky of A~^T A~ alone (its
 * factor is the QRCP factor with positive diagonal; in floating point it
 * decides residual norms down to about sqrt(u) R_00 ~ 1.5e-8 R_00 and its
 * R carries relative error about u kappa(R11)^2).  For 1e-10 <= zeta < 1e-5
 * a refinement: the Gram pivoting down to 1e-5 R_00, those columns
 * orthonormalised by Cholesky QR twice and projected out of the others
 * twice, pivoting again on the Gram of that explicit residual (cutoff
 * zeta R_00), Cholesky QR twice of the new columns, and R's rows as Q^T A~;
 * rank, pivots (off near-ties) and R (to rounding, relative error about
 * u kappa(R11)) are those of Householder QRCP on A~.  zeta < 1e-10 gives
 * LEV_ERR_NOT_SUPPORTED.  Requires d <= 1024 and d <= m. */
lev_status lev_rank_estimate(const double* At, int64_t m, int64_t d, double zeta,
                             int32_t* perm_out, double* R_out, int64_t* rank_out,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 10 (LS-HRN-approx): sketch, rank-revealing QR, then Algorithm 8
 * on the selected columns K = perm[0..r): theta~_i = || A[i, K] Z ||^2 with
 * Z = R11^{-1} G_k[0:r, :], R11 the leading r x r block of R and G_k the
 * d x k JL Gaussian scaled by 1/sqrt(k) (row j of G_k pairs with pivot
 * position j).
 *  theta_out -- n entries: FP64 when A is F64, else FP32.
 *  state_out -- optional (NULL to skip): lev_state_size(d, m, k) bytes that
 *               lev_estimate_backward needs (perm, rank, R, Z, A~); 256-byte
 *               aligned.  Its header is int64[8]: [0] a magic value, [1] d,
 *               [2] m, [3] k, [4] the rank r, [5] the device error word (low
 *               32 bits; 0 on success).  The kernels' waits on each other
 *               end by construction but are bounded; a wait that ran out sets
 *               bit 1 (pivoting) or bit 2 (triangular solve) of the error
 *               word, and the call's results are then meaningless.  The word
 *               is cleared at the start of every call.
 * Dense (F64/F32/BF16) and CSR (F64/F32/BF16 values) input.
 * r = 0 (e.g. A = 0) gives theta~ = 0.  Zero rows give theta~_i = 0. */
lev_status lev_estimate(const lev_matrix* A, const lev_params* p, void* theta_out,
                        void* state_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* lev_estimate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and the same kernels, with the workspace taken from a
 * static device array of lev_noalloc_max_bytes() bytes (64 MiB) inside the
 * library instead of a caller buffer, and no state output.  The call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * the array is part of the library's device code and each GPU the call runs
 * on holds its own copy from the first call on that GPU until the process
 * ends.  The current device must be the device of A, theta_out and stream.
 *  Returns LEV_ERR_WORKSPACE, before touching the device, when
 *  lev_workspace_size(A, p, LEV_WS_ESTIMATE) exceeds the array (e.g. the
 *  Gaussian G_m of an m x r_cs sketch above about 5e6 elements).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from different host threads with different
 * streams) race and give wrong results; calls on one stream are ordered and
 * safe.  Each call clears what it needs cleared. */
size_t lev_noalloc_max_bytes(void);
lev_status lev_estimate_noalloc(const lev_matrix* A, const lev_params* p, void* theta_out, hipStream_t stream);

/* Adjoint of f(A) = sum_i w_i theta~_i with the sketch (S, G_m, G_k), the
 * pivots K and the rank r held fixed (the paper differentiates nothing; this
 * is the reverse of Algorithms 3, 4 and 8 step by step):
 *   Y = A_K Z,  C = A_K^T diag(w) Y,  Zbar = 2 C,
 *   Rbar = -triu(R11^{-T} Zbar Z^T),  A~_K bar = Q copyltu(R11 Rbar^T) R11^{-T}
 *   (Q = A~_K R11^{-1}),  H = G^T A~_K bar,
 *   gradA[i, K] = 2 w_i Y_i Z^T + s_i H[h(i), :],  gradA[i, not K] = 0.
 *  A         -- the same dense matrix lev_estimate saw (F32 or F64 only;
 *               CSR gives LEV_ERR_NOT_SUPPORTED, BF16 LEV_ERR_DTYPE).
 *  p         -- the same parameters.
 *  state     -- the blob lev_estimate wrote for this A and p (256-byte
 *               aligned); it is read, and only its error word (header slot
 *               5) may be written: a bounded wait of the triangular solve
 *               that ran out sets bit 2 there.  A blob from another A
 *               or other parameters gives a meaningless gradient (its header
 *               is not checked on the host, which would need a sync).
 *  w         -- n weights of A's type.
 *  gradA_out -- n x ld, A's type; columns >= d are not written.
 * Workspace: lev_workspace_size(A, p, LEV_WS_BACKWARD).  Two passes over A
 * (Y is recomputed in each, never stored), FP64 for the d x d core. */
lev_status lev_estimate_backward(const lev_matrix* A, const lev_params* p, const void* state,
                                 const void* w, void* gradA_out, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

/* ---- least squares (Section 6) ----------------------------------------------- */

/* Algorithm 11 (CountGaussPrecondition): a right preconditioner N for
 * min ||A x - b|| from the same sketch and rank-revealing step as
 * lev_estimate (p's seed, r_cs, m, zeta and sketch; k, mode and
 * az_precision unused).  With A~ P = Q R the factor of the sketch:
 *  method LEV_PRECOND_QR:  N = P R11^{-1}, k = the rank r;
 *  method LEV_PRECOND_SVD: N = V_k Sigma_k^{-1} from the SVD of A~ (taken
 *    as the SVD of R by one-sided Jacobi, so d <= 128, else
 *    LEV_ERR_NOT_SUPPORTED), k = #{ sigma_j > zeta sigma_1 }.
 * N_out: d x d FP64 row-major (device), columns >= k zero; k_out: int64
 * (device), -1 when a bounded wait of the rank-revealing step ran out.
 * The section's theorem bounds kappa(A N) by ((1 + alpha + sqrt(k/m)) /
 * (1 - alpha - sqrt(k/m))) ((1 + eps) / (1 - eps)) with high probability,
 * whatever kappa(A).  Workspace: lev_precondition_workspace_size. */
enum { LEV_PRECOND_QR = 0, LEV_PRECOND_SVD = 1 };
size_t lev_precondition_workspace_size(const lev_matrix* A, const lev_params* p);
lev_status lev_precondition(const lev_matrix* A, const lev_params* p, int method, double* N_out, int64_t* k_out,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* LSQR (Paige and Saunders) on the preconditioned operator A N from y = 0,
 * iters steps, x_out = N y (d, FP64, device): with N from lev_precondition,
 * x approaches A^+ b (SVD) or a least-squares solution (QR).  A dense
 * (any dtype; the arithmetic is FP64), N d x d FP64 (device), b n FP64
 * (device), resid_out (device, may be NULL): the residual-norm estimate
 * ||A x_t - b|| after each step t < iters.  The steps stop early (the later
 * entries repeat the last estimate) if the bidiagonalisation breaks down
 * exactly (alpha or beta = 0).  Two passes over A per step.  CSR gives
 * LEV_ERR_NOT_SUPPORTED.  Workspace: lev_lsqr_workspace_size. */
size_t lev_lsqr_workspace_size(const lev_matrix* A);
lev_status lev_lsqr(const lev_matrix* A, const double* N, const double* b, int64_t iters, double* x_out,
                    double* resid_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- inspection helpers (used by the tests) -------------------------------- */

/* Host-only: the CountSketch hash and sign coefficients a seed expands to
 * (Section 3.4, CountSketch: a pairwise independent bucket hash and 4-wise
 * independent signs).  out (HOST, 7 entries) receives P (the smallest prime
 * >= max(n, 2)), a and c of h(i) = ((a i + c) mod P) mod r_cs, and c0..c3 of
 * the sign polynomial (c3 i^3 + c2 i^2 + c1 i + c0) mod (2^61 - 1).  No
 * device work; callable without a GPU. */
lev_status lev_hash_params(uint64_t seed, int64_t n, int64_t r_cs, uint64_t* out);

/* h(i) and s(i) of the CountSketch for every row i < n (int64 h_out[n],
 * int8 s_out[n], device). */
lev_status lev_debug_hash(uint64_t seed, int64_t n, int64_t r_cs, int64_t* h_out,
                          int8_t* s_out, hipStream_t stream);

/* S in compressed form, as pass 1 enumerates it: bucket_off int64[r_cs+1]
 * and bucket_rows int32[n] (rows of bucket b in bucket_rows[bucket_off[b] ..
 * bucket_off[b+1]), in the order pass 1 accumulates them). */
lev_status lev_debug_buckets(uint64_t seed, int64_t n, int64_t r_cs, int64_t* bucket_off,
                             int32_t* bucket_rows, hipStream_t stream);

/* The Gaussian matrices of a seed: which = 0 -> G_m / sqrt(m) (rows = m,
 * cols = r_cs), which = 1 -> G_k / sqrt(k) (rows = d, cols = k).  out is
 * rows x cols FP64 row-major. */
lev_status lev_debug_gaussian(uint64_t seed, int which, int64_t rows, int64_t cols,
                              double* out, hipStream_t stream);

/* The read ceiling the passes over A are measured against: reads `bytes`
 * of device memory at buf (16-byte aligned, bytes a multiple of 16) once,
 * with 16-byte loads from 256 workgroups of 1024 threads, and stores one
 * checksum per thread into sink (device, LEV_STREAM_READ_SINK uint32; the
 * XOR of all of them is the XOR over the 16-byte vectors of the sum of
 * their four 32-bit words, mod 2^32).  Nothing else is read or written.
 * LEV_ERR_ARG for a null pointer, misaligned buf or bytes not a positive
 * multiple of 16. */
#define LEV_STREAM_READ_SINK 262144
lev_status lev_debug_stream_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t stream);

/* Phase timing.  Registers `count` caller-created HIP events (count must be
 * LEV_PHASES, or 0 / NULL to stop) for the calling thread; each following
 * lev_estimate call on that thread records them on its stream at the phase
 * boundaries: [0] start, [1] before pass 1 (nothing runs in between: the
 * Gaussian draws run inside pass 1), [2] after pass 1 (S A and the draws),
 * [3] after A~ = G (S A), [4] after the rank-revealing factorisation,
 * [5] after Z is formed, [6] after pass 2 (theta~).  The events stay owned
 * by the caller. */
#define LEV_PHASES 7
lev_status lev_set_phase_events(hipEvent_t* events, int count);

const char* lev_status_string(lev_status s);
const char* lev_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LEV_H */
