"""Reference gradient of f(A) = sum_i w_i theta~_i(A) at a fixed sketch.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper differentiates nothing; this is the adjoint of its estimator
(Algorithm 10) with every random object (S, G, Pi_2) and the discrete
choices (the pivots K and the rank r) held fixed, so f is a smooth function
of A around a point where the pivoting does not change.  Forward, in the
order of Algorithms 3, 4 and 8:

    SA  = S A                       (CountSketch, Section 3.4)
    A~  = G (S A)                   (Algorithm 3)
    Q R = A~[:, K]                  (Algorithm 8, step 3; diag(R) > 0)
    Z   = R^{-1} Pi_2[:r]           (Algorithm 8, step 4)
    Y   = A[:, K] Z,  theta~_i = ||Y_i||^2      (Algorithm 8, step 5)
    f   = sum_i w_i theta~_i

Reverse, each step's adjoint in turn (bars are df/d(.)):

    Ybar        = 2 diag(w) Y
    A[:, K]bar  = Ybar Z^T                      (through Y = A_K Z)
    Zbar        = A_K^T Ybar
    Rbar        = -triu(R^{-T} Zbar Z^T)        (Z = R^{-1} Pi_2, R upper)
    A~_K bar    = Q copyltu(R Rbar^T) R^{-T}    (QR with R upper, Q fixed
                  columns' span; copyltu(M) = tril(M) + tril(M, -1)^T)
    (SA)_K bar  = G^T A~_K bar
    A[:, K]bar += S^T (SA)_K bar,   i.e. row i gets s_i (SA)_K bar[h(i), :]
    A[:, not K]bar = 0

The QR adjoint is the standard one for A = QR with a square upper
triangular R of positive diagonal.  The tests pin this module against
central finite differences and against an independent autograd route.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import conventions as conv
from . import leverage as L


@dataclass
class Gradient:
    f: float
    theta: np.ndarray
    grad: np.ndarray      # n x d
    perm: np.ndarray
    rank: int


def copyltu(M: np.ndarray) -> np.ndarray:
    """The lower triangle of M mirrored onto the upper one."""
    return np.tril(M) + np.tril(M, -1).T


def countsketch_transpose_apply(rnd: conv.SketchRandomness, X: np.ndarray) -> np.ndarray:
    """S^T X for the CountSketch S (r_cs x n): row i is s_i X[h(i), :]."""
    h, s = conv.buckets(rnd), conv.signs(rnd)
    return s[:, None] * X[h, :]


def estimate_and_gradient(A: np.ndarray, seed: int, r_cs: int, m: int, k_jl: int, zeta: float,
                          w: np.ndarray, perm=None, rank=None) -> Gradient:
    """f = w^T theta~ and df/dA (dense FP64).  The pivots and rank come from
    the oracle's own QRCP of the sketch unless given (finite differences
    pass them in so that they stay fixed)."""
    A = np.asarray(A, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d = A.shape
    rnd = conv.derive(seed, n, r_cs)
    # forward
    SA = L.countsketch_apply(rnd, A)
    Gm = conv.gaussian_transform(rnd, m)
    At = Gm @ SA
    if perm is None or rank is None:
        rr = L.qrcp_sign_normalised(At, zeta)
        perm, rank = rr.perm, rr.rank
    perm = np.asarray(perm, dtype=np.int64)
    r = int(rank)
    grad = np.zeros((n, d))
    if r == 0:
        return Gradient(0.0, np.zeros(n), grad, perm, 0)
    K = perm[:r]
    Q, R = np.linalg.qr(At[:, K], mode="reduced")
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    Q, R = Q * sgn[None, :], R * sgn[:, None]
    Pi2 = conv.jl_gaussian(rnd, d, k_jl)[:r]
    Z = sla.solve_triangular(R, Pi2, lower=False)
    AK = A[:, K]
    Y = AK @ Z
    theta = np.sum(Y * Y, axis=1)
    f = float(w @ theta)
    # reverse
    Ybar = 2.0 * w[:, None] * Y
    AK_bar = Ybar @ Z.T
    Zbar = AK.T @ Ybar
    Rbar = -np.triu(sla.solve_triangular(R, Zbar @ Z.T, lower=False, trans="T"))
    Mq = copyltu(R @ Rbar.T)
    AtK_bar = sla.solve_triangular(R, (Q @ Mq).T, lower=False).T  # (Q Mq) R^{-T}
    SAK_bar = Gm.T @ AtK_bar
    AK_bar = AK_bar + countsketch_transpose_apply(rnd, SAK_bar)
    grad[:, K] = AK_bar
    return Gradient(f, theta, grad, perm, r)
