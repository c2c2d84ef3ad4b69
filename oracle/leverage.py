"""Leverage scores, exact and estimated, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Exact scores (Section 1): theta_i is the i-th diagonal entry of the hat
matrix H = A (A^T A)^+ A^T, equivalently the squared norm of row i of any
orthonormal basis of range(A) (H is the unique orthogonal projector onto
range(A)).  The routes below are independent computations of that one
quantity and the tests check them against each other.

Estimator LS-HRN-approx (Algorithm 10):
  1. Algorithm 4 (CountGaussSRRQR): sketch A~ = G (S A) (Algorithm 3), then a
     rank-revealing QR of A~ giving the permutation P_k, R_k and the rank k.
     The paper's implementation replaces the strong RRQR by the classical
     column-pivoted QR of LAPACK xGEQP3 (Section 7); so does this oracle,
     through scipy.linalg.qr(pivoting=True), which calls DGEQP3.
  2. Keep A_{:,K} = A P_k.
  3. Algorithm 8 on A_{:,K} with Pi_1 = G S (or F S, the SRHT composition of
     Section 4): R~ from a QR of Pi_1 A_{:,K},
     X = R~^{-1} Pi_2, theta~_i = ||e_i^T A_{:,K} X||^2.

Readings of points the paper leaves open (listed with their reasons in the
design notes of the repository):
  * G is scaled by 1/sqrt(m) and Pi_2 by 1/sqrt(k) (Gaussian embeddings,
    Section 3.4); the bare N(0,1) of Algorithm 3 would scale theta~ by 1/m.
  * R is sign-normalised to a non-negative diagonal (the QR factor with a
    positive diagonal is unique; Z = R^{-1} Pi_2 depends on the signs).
  * Rank rule: k = #{ j : R_jj > zeta * R_00 } on the normalised QRCP
    diagonal, the cutoff test of Section 7 (|R~_kk| < c |R~_11|).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import conventions as conv


# ==========================================================================
# Exact leverage scores
# ==========================================================================
def exact_theta_svd(A: np.ndarray, tol: float) -> tuple[np.ndarray, int]:
    """theta_i = sum_{j <= rho} U_ij^2 from the thin SVD A = U S V^T, with
    the numerical rank rho = #{ sigma_j > tol * sigma_1 } (Section 1: row
    norms of an orthonormal basis of range(A))."""
    A = np.asarray(A, dtype=np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros(A.shape[0]), 0
    rho = int(np.sum(s > tol * s[0]))
    return np.sum(U[:, :rho] ** 2, axis=1), rho


def hat_diagonal_bruteforce(A: np.ndarray, tol: float) -> np.ndarray:
    """diag(A (A^T A)^+ A^T), the hat-matrix definition of Section 1 written
    out literally (forms the n x n matrix: small n only).  The pseudoinverse
    drops eigenvalues of A^T A below tol^2 * lambda_max, i.e. singular values
    of A below tol * sigma_1."""
    A = np.asarray(A, dtype=np.float64)
    gram = A.T @ A
    pinv = np.linalg.pinv(gram, rcond=tol ** 2, hermitian=True)
    H = A @ pinv @ A.T
    return np.diag(H).copy()


def theta_householder_qr(A: np.ndarray) -> np.ndarray:
    """Q, R = qr(A); theta = sum(Q .* Q, dims=2) -- the QR one-liner of
    Section 1 (valid for full column rank A)."""
    Q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    return np.sum(Q * Q, axis=1)


def theta_least_squares(A: np.ndarray) -> np.ndarray:
    """theta_i = ||e_i^T A X||^2 with X = argmin_Y ||A Y - I_n||_F (the least
    squares form of Section 1; small n only)."""
    A = np.asarray(A, dtype=np.float64)
    X, *_ = np.linalg.lstsq(A, np.eye(A.shape[0]), rcond=None)
    return np.sum((A @ X) ** 2, axis=1)


def theta_gram(A, tol: float) -> tuple[np.ndarray, int]:
    """Algorithm 5 (Gram pseudoinverse): B = A^T A as a sum of row outer
    products (Lemma on the Gram complexity), B = V S^2 V^T, keep the rank-k
    part, theta_i = ||e_i^T A V_k S_k^{-1}||^2.  Accepts dense or scipy
    sparse A."""
    if sp.issparse(A):
        A = A.tocsr().astype(np.float64)
        B = (A.T @ A).toarray()
    else:
        A = np.asarray(A, dtype=np.float64)
        B = A.T @ A
    w, V = np.linalg.eigh(B)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    sig = np.sqrt(np.clip(w, 0.0, None))
    if sig.size == 0 or sig[0] == 0.0:
        return np.zeros(A.shape[0]), 0
    k = int(np.sum(sig > tol * sig[0]))
    W = V[:, :k] / sig[:k]
    Y = A @ W
    Y = np.asarray(Y)
    return np.sum(Y * Y, axis=1), k


def theta_gram_rows(chunks, rows, tol: float) -> tuple[np.ndarray, int]:
    """Algorithm 5 for a matrix too large to hold at once: ``chunks`` is a
    callable returning an iterable of (row offset, FP64 block of consecutive
    rows) covering A in order (it is called twice).  Pass 1 accumulates
    B = A^T A block by block; B = V S^2 V^T keeps the rank-k part
    (S_jj > tol * S_11); pass 2 returns theta_i = ||e_i^T A V_k S_k^{-1}||^2
    for the sorted row indices ``rows`` only.  Returns (theta[rows], k)."""
    rows = np.asarray(rows, dtype=np.int64)
    B = None
    for _, blk in chunks():
        blk = np.asarray(blk, dtype=np.float64)
        B = blk.T @ blk if B is None else B + blk.T @ blk
    w, V = np.linalg.eigh(B)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    sig = np.sqrt(np.clip(w, 0.0, None))
    out = np.zeros(rows.size)
    if sig.size == 0 or sig[0] == 0.0:
        return out, 0
    k = int(np.sum(sig > tol * sig[0]))
    W = V[:, :k] / sig[:k]
    for lo, blk in chunks():
        hi = lo + blk.shape[0]
        sel = (rows >= lo) & (rows < hi)
        if np.any(sel):
            Y = np.asarray(blk, dtype=np.float64)[rows[sel] - lo] @ W
            out[sel] = np.sum(Y * Y, axis=1)
    return out, k


# ==========================================================================
# Algorithm 3: CountGaussSketch
# ==========================================================================
def countsketch_dense_S(rnd: conv.SketchRandomness) -> np.ndarray:
    """S as a dense r_cs x n matrix: S[h(i), i] = s(i) (tiny n only)."""
    S = np.zeros((rnd.r_cs, rnd.n))
    for i in range(rnd.n):
        S[conv.bucket_of(rnd, i), i] = conv.sign_of(rnd, i)
    return S


def countsketch_apply(rnd: conv.SketchRandomness, A, chunk: int = 1 << 16) -> np.ndarray:
    """S A (r_cs x d, FP64), with S the CountSketch of Section 3.4, applied
    as a sparse matrix over row chunks of A (dense ndarray or scipy sparse)."""
    h, cols, s = conv.countsketch_matrix_entries(rnd)
    S = sp.csc_matrix((s, (h, cols)), shape=(rnd.r_cs, rnd.n))  # column slices below
    d = A.shape[1]
    SA = np.zeros((rnd.r_cs, d))
    for lo in range(0, rnd.n, chunk):
        hi = min(rnd.n, lo + chunk)
        blk = A[lo:hi]
        if sp.issparse(blk):
            SA += np.asarray((S[:, lo:hi] @ blk.astype(np.float64)).todense())
        else:
            SA += S[:, lo:hi] @ np.asarray(blk, dtype=np.float64)
    return SA


def fwht(X: np.ndarray) -> np.ndarray:
    """H X for the unscaled Walsh-Hadamard matrix of Sylvester order
    (H[i][j] = (-1)^popcount(i & j)), along axis 0 (length a power of two),
    by the butterflies (a, b) -> (a + b, a - b) over each bit."""
    Y = np.array(X, dtype=np.float64, copy=True)
    r = Y.shape[0]
    h = 1
    while h < r:
        Y = Y.reshape(r // (2 * h), 2, h, *Y.shape[1:])
        a, b = Y[:, 0].copy(), Y[:, 1].copy()
        Y[:, 0], Y[:, 1] = a + b, a - b
        Y = Y.reshape(r, *Y.shape[3:])
        h *= 2
    return Y


def srht_apply(rnd: conv.SketchRandomness, SA: np.ndarray, t: int) -> np.ndarray:
    """F (S A) for the SRHT F = sqrt(r / t) P (H / sqrt(r)) D of Section 3.4
    (= P H D / sqrt(t) with the unscaled H): D's signs, then H (the dense
    Sylvester matrix of scipy for r <= 4096, the butterflies above beyond),
    then rows pi(0), ..., pi(t - 1)."""
    r = SA.shape[0]
    D = np.array([conv.srht_sign(rnd, j) for j in range(r)], dtype=np.float64)
    X = D[:, None] * SA
    HX = sla.hadamard(r) @ X if r <= 4096 else fwht(X)
    rows = [conv.srht_coordinate(rnd, r, j) for j in range(t)]
    return HX[rows] / math.sqrt(t)


SKETCHES = ("gauss", "srht")


def count_gauss_sketch(rnd: conv.SketchRandomness, A, m: int, sketch: str = "gauss"):
    """Algorithm 3: A~ = G (S A), with G = G_m / sqrt(m).  sketch="srht":
    A~ = F (S A) with the m x r_cs SRHT F in place of G (the F S composition
    of Section 4).  Returns (A~, SA)."""
    if sketch not in SKETCHES:
        raise ValueError(f"sketch must be one of {SKETCHES}")
    SA = countsketch_apply(rnd, A)
    if sketch == "srht":
        return srht_apply(rnd, SA, m), SA
    G = conv.gaussian_transform(rnd, m)
    return G @ SA, SA


# ==========================================================================
# Algorithm 4: CountGaussSRRQR (QRCP in place of SRRQR, as in Section 7)
# ==========================================================================
@dataclass
class RankRevealing:
    perm: np.ndarray      # int64[d]: column j of A~ P is column perm[j] of A~
    R: np.ndarray         # d x d upper triangular, non-negative diagonal
    rank: int             # k = #{ j : R_jj > zeta R_00 }


def qrcp_sign_normalised(At: np.ndarray, zeta: float) -> RankRevealing:
    """Column-pivoted QR of A~ (LAPACK DGEQP3, the routine of Section 7),
    R's rows flipped so diag(R) >= 0, and the cutoff rank rule."""
    At = np.asarray(At, dtype=np.float64)
    _, R, perm = sla.qr(At, mode="economic", pivoting=True)
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    R = R * sgn[:, None]
    dg = np.diag(R)
    if dg.size == 0 or dg[0] <= 0.0:
        rank = 0
    else:
        rank = int(np.sum(dg > zeta * dg[0]))
    return RankRevealing(np.asarray(perm, dtype=np.int64), R, rank)


def count_gauss_srrqr(rnd: conv.SketchRandomness, A, m: int, zeta: float, sketch: str = "gauss"):
    """Algorithm 4: returns (P_k as column ids, R_k, k) plus the sketch."""
    At, SA = count_gauss_sketch(rnd, A, m, sketch)
    rr = qrcp_sign_normalised(At, zeta)
    k = rr.rank
    return rr.perm[:k], rr.R[:k, :k], k, At, SA, rr


# ==========================================================================
# Algorithm 8 on A_{:,K}, and Algorithm 10
# ==========================================================================
def r_from_qr_of_sketch(AtK: np.ndarray) -> np.ndarray:
    """Algorithm 8 step 3 with Pi_1 = G S: R~ from an (unpivoted) QR of
    Pi_1 A_{:,K} = A~[:, K], sign-normalised to a non-negative diagonal."""
    _, R = np.linalg.qr(AtK, mode="reduced")
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return R * sgn[:, None]


def jl_orthogonalizer(R: np.ndarray, Pi2: np.ndarray) -> np.ndarray:
    """Algorithm 8 step 4: X = R~^{-1} Pi_2 (back substitution)."""
    return sla.solve_triangular(R, Pi2, lower=False)


def row_norms_sq(AK, X: np.ndarray, rows=None, chunk: int = 1 << 16) -> np.ndarray:
    """Algorithm 8 step 5: theta~_i = ||e_i^T A_{:,K} X||^2 (rows subset
    optional)."""
    if rows is not None:
        blk = AK[rows]
        Y = blk @ X
        Y = np.asarray(Y.todense() if sp.issparse(Y) else Y)
        return np.sum(Y * Y, axis=1)
    n = AK.shape[0]
    out = np.empty(n)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        blk = AK[lo:hi]
        if sp.issparse(blk):
            Y = np.asarray(blk.astype(np.float64) @ X)
        else:
            Y = np.asarray(blk, dtype=np.float64) @ X
        out[lo:hi] = np.sum(Y * Y, axis=1)
    return out


@dataclass
class Estimate:
    theta: np.ndarray | None   # theta~ (None when only sampled rows were asked)
    theta_rows: np.ndarray | None
    perm: np.ndarray           # full QRCP permutation of the sketch
    rank: int
    R11: np.ndarray            # k x k orthogonalizer R~ of A_{:,K}
    Z: np.ndarray              # X = R~^{-1} Pi_2, k x k_jl
    At: np.ndarray             # A~ = G S A
    SA: np.ndarray
    R_full: np.ndarray         # sign-normalised QRCP R of A~
    G_k: np.ndarray            # d x k_jl JL Gaussian (rows used: 0..rank-1)


def ls_hrn_approx(A, seed: int, r_cs: int, m: int, k_jl: int, zeta: float, rows=None,
                  sketch: str = "gauss") -> Estimate:
    """Algorithm 10 (LS-HRN-approx) with the readings listed in the module
    docstring.  ``rows`` restricts the final row-norm step to a subset (the
    sketch still uses all of A); sketch="srht" takes Pi_1 = F S."""
    n, d = A.shape
    rnd = conv.derive(seed, n, r_cs)
    K, _, k, At, SA, rr = count_gauss_srrqr(rnd, A, m, zeta, sketch)
    Gk = conv.jl_gaussian(rnd, d, k_jl)
    if k == 0:
        th = np.zeros(n) if rows is None else None
        thr = np.zeros(len(rows)) if rows is not None else None
        return Estimate(th, thr, rr.perm, 0, np.zeros((0, 0)), np.zeros((0, k_jl)), At, SA, rr.R, Gk)
    R11 = r_from_qr_of_sketch(At[:, K])
    Z = jl_orthogonalizer(R11, Gk[:k])
    if rows is None:
        return Estimate(row_norms_sq(A[:, K], Z), None, rr.perm, k, R11, Z, At, SA, rr.R, Gk)
    AK_rows = A[np.asarray(rows)][:, K]
    return Estimate(None, row_norms_sq(AK_rows, Z), rr.perm, k, R11, Z, At, SA, rr.R, Gk)


@dataclass
class ExactEstimate:
    theta: np.ndarray | None
    theta_rows: np.ndarray | None
    perm: np.ndarray           # full QRCP permutation of the sketch
    rank: int


def ls_hrn_exact(A, seed: int, r_cs: int, m: int, zeta: float, rows=None, sketch: str = "gauss") -> ExactEstimate:
    """Algorithm 7 (LS-HRN-exact): the columns K and the rank k from
    Algorithm 4 on the sketch (as in ls_hrn_approx), then B = A_K^T A_K, its
    eigendecomposition B = V Sigma^2 V^T (the SVD of a symmetric positive
    definite B), and theta~_i = ||e_i^T A_K V Sigma^{-1}||^2: the exact
    leverage scores of A_K.  ``rows`` restricts the last step to a subset."""
    n, d = A.shape
    rnd = conv.derive(seed, n, r_cs)
    K, _, k, _, _, rr = count_gauss_srrqr(rnd, A, m, zeta, sketch)
    if k == 0:
        return ExactEstimate(np.zeros(n) if rows is None else None,
                             np.zeros(len(rows)) if rows is not None else None, rr.perm, 0)
    AK = A[:, K]
    if sp.issparse(AK):
        AK = AK.tocsr().astype(np.float64)
        B = (AK.T @ AK).toarray()
    else:
        AK = np.asarray(AK, dtype=np.float64)
        B = AK.T @ AK
    w, V = np.linalg.eigh(B)
    W = V / np.sqrt(w)  # V Sigma^{-1}
    th = row_norms_sq(AK, W, rows=rows)
    if rows is None:
        return ExactEstimate(th, None, rr.perm, k)
    return ExactEstimate(None, th, rr.perm, k)


def theta_prime(A, K: np.ndarray, R11: np.ndarray, rows=None) -> np.ndarray:
    """The estimate without the JL step: ||e_i^T A_{:,K} R~^{-1}||^2."""
    X = sla.solve_triangular(R11, np.eye(R11.shape[0]), lower=False)
    return row_norms_sq(A[:, K], X, rows=rows)


# ==========================================================================
# Algorithm 6: exact scores from a Q-less sparse pivoted QR
# ==========================================================================
@dataclass
class QlessQR:
    perm: np.ndarray   # the k pivots, in order
    R: np.ndarray      # k x k upper triangular, positive diagonal: (A P_k)^T (A P_k) = R^T R
    rank: int


def qless_pivoted_qr(A, zeta: float, max_rank: int) -> QlessQR:
    """Algorithm 6 step 1: column-pivoted Gram-Schmidt without Q (the SPQR of
    Berry, Pulatova and Stewart that Section 5 adopts).  Q_j = A_K R^{-1}
    stays implicit: step j takes the column p of largest remaining norm^2
    s_p (s_c = ||a_c||^2 minus the squares of its R entries so far), sets
    r_jj = sqrt(s_p) and, from the inner products b = A^T a_p,
    r_jc = (b_c - sum_{i<j} r_ip r_ic) / r_jj, then s_c -= r_jc^2.  It stops
    at max_rank steps, or before a step with r_jj <= zeta * r_00 (the rank
    rule of Section 7).  Ties in the norm go to the lowest column."""
    d = A.shape[1]
    if sp.issparse(A):
        A = A.tocsc().astype(np.float64)
        s = np.asarray(A.multiply(A).sum(axis=0)).ravel()

        def AtA_col(p):
            return np.asarray((A.T @ A[:, [p]]).todense()).ravel()
    else:
        A = np.asarray(A, dtype=np.float64)
        s = np.einsum("ij,ij->j", A, A)

        def AtA_col(p):
            return A.T @ A[:, p]
    rows = np.zeros((0, d))
    chosen: list[int] = []
    r00 = 0.0
    for j in range(min(max_rank, d)):
        cand = [c for c in range(d) if c not in chosen]
        p = max(cand, key=lambda c: (s[c], -c))
        rjj = math.sqrt(max(s[p], 0.0))
        if j == 0:
            r00 = rjj
        if rjj <= 0.0 or rjj <= zeta * r00:
            break
        b = AtA_col(p)
        row = (b - rows[:, p] @ rows) / rjj
        row[p] = rjj
        row[chosen] = 0.0
        for c in cand:
            if c != p:
                s[c] -= row[c] ** 2
        rows = np.vstack([rows, row])
        chosen.append(p)
    k = len(chosen)
    perm = np.asarray(chosen, dtype=np.int64)
    return QlessQR(perm, rows[:, perm] if k else np.zeros((0, 0)), k)


def ls_qless_qr(A, zeta: float, max_rank: int, rows=None) -> tuple[np.ndarray, QlessQR]:
    """Algorithm 6: theta_i = ||e_i^T A P_k R_k^{-1}||^2 with P_k, R_k from
    the Q-less pivoted QR above (no sketch)."""
    qr = qless_pivoted_qr(A, zeta, max_rank)
    n = A.shape[0]
    if qr.rank == 0:
        return np.zeros(n if rows is None else len(rows)), qr
    X = sla.solve_triangular(qr.R, np.eye(qr.rank), lower=False)
    AK = A[:, qr.perm]
    return row_norms_sq(AK, X, rows=rows), qr


def qrcp_reference_small(At: np.ndarray) -> np.ndarray:
    """Businger-Golub column pivoting written out (tiny inputs): at each step
    the pivot is the remaining column of largest residual norm, recomputed
    exactly by projecting out the columns already chosen.  Returns the
    permutation; used to pin the LAPACK route."""
    At = np.asarray(At, dtype=np.float64)
    d = At.shape[1]
    chosen: list[int] = []
    Q = np.zeros((At.shape[0], 0))
    for _ in range(d):
        best, best_norm = -1, -1.0
        for c in range(d):
            if c in chosen:
                continue
            resid = At[:, c] - Q @ (Q.T @ At[:, c])
            nrm = float(resid @ resid)
            if nrm > best_norm:
                best, best_norm = c, nrm
        chosen.append(best)
        resid = At[:, best] - Q @ (Q.T @ At[:, best])
        nr = math.sqrt(max(best_norm, 0.0))
        q = resid / nr if nr > 0 else resid * 0.0
        Q = np.column_stack([Q, q])
    return np.asarray(chosen, dtype=np.int64)
