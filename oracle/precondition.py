"""Right preconditioning of tall least-squares problems (Section 6) and the
LSQR solver that uses it, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 11 (CountGaussPrecondition): sketch A~ = G (S A) (Algorithm 3),
take the SVD A~ = U Sigma V^T, keep the k singular values above zeta times
the largest, and return N = V_{:,1:k} Sigma_{1:k}^{-1}.  The section's
theorem bounds kappa(A N) by xi * eta with high probability, independently
of kappa(A), and N y-hat = A^+ b for the minimum-length y-hat of
min ||A N y - b||.  The experiments also build N from the pivoted QR of the
sketch, N = P_k R_k^{-1}; both are written out here.

Reading: the rank rule of the algorithm's third step is garbled in the
text (an argmax over sigma_j with sigma_j / sigma_1 <= zeta); it is read as
k = #{ j : sigma_j > zeta sigma_1 }, the cutoff rule used everywhere else.

LSQR (Paige and Saunders, ACM TOMS 8(1), 1982): the Golub-Kahan
bidiagonalisation of the operator M = A N started from b, with the
QR-updated iterate, written from that paper's recurrences; the iterate in
the preconditioned space is mapped back by x = N y.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import conventions as conv
from . import leverage as L


def count_gauss_precondition(A, seed: int, r_cs: int, m: int, zeta: float, method: str = "svd",
                             sketch: str = "gauss") -> tuple[np.ndarray, int]:
    """Algorithm 11: (N, k) with N d x k.  method="qr": N = P_k R_k^{-1}
    from the sign-normalised column-pivoted QR of the sketch."""
    n, d = A.shape
    rnd = conv.derive(seed, n, r_cs)
    At, _ = L.count_gauss_sketch(rnd, A, m, sketch)
    if method == "svd":
        _, s, Vt = np.linalg.svd(At, full_matrices=False)
        k = int(np.sum(s > zeta * s[0])) if s.size and s[0] > 0 else 0
        return Vt[:k].T / s[:k], k
    rr = L.qrcp_sign_normalised(At, zeta)
    k = rr.rank
    N = np.zeros((d, k))
    N[rr.perm[:k]] = sla.solve_triangular(rr.R[:k, :k], np.eye(k), lower=False)
    return N, k


def kappa_bound(k: int, m: int, alpha: float, eps: float) -> float:
    """xi * eta of the preconditioning theorem of Section 6."""
    t = math.sqrt(k / m)
    return (1 + alpha + t) / (1 - alpha - t) * (1 + eps) / (1 - eps)


def lsqr(matvec, rmatvec, b: np.ndarray, iters: int) -> tuple[np.ndarray, list[float]]:
    """``iters`` steps of LSQR on min ||M y - b|| (M given by y -> M y and
    u -> M^T u), from y = 0.  Returns y and the residual-norm estimates
    phi-bar after each step."""
    u = np.array(b, dtype=np.float64)
    beta = float(np.linalg.norm(u))
    if beta > 0:
        u = u / beta
    v = rmatvec(u)
    alpha = float(np.linalg.norm(v))
    if alpha > 0:
        v = v / alpha
    w = v.copy()
    y = np.zeros_like(v)
    phibar, rhobar = beta, alpha
    hist = []
    for _ in range(iters):
        if alpha == 0.0 or beta == 0.0:
            hist.append(phibar)
            continue
        u = matvec(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u = u / beta
        v = rmatvec(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v = v / alpha
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        hist.append(phibar)
    return y, hist


def preconditioned_lsqr(A, N: np.ndarray, b: np.ndarray, iters: int) -> tuple[np.ndarray, list[float]]:
    """LSQR on A N, then x = N y (the solution of Section 6's theorem)."""
    A = A.astype(np.float64) if hasattr(A, "astype") else np.asarray(A, dtype=np.float64)
    y, hist = lsqr(lambda z: A @ (N @ z), lambda r: N.T @ (A.T @ r), b, iters)
    return N @ y, hist
