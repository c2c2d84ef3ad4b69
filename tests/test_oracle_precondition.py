"""Pins of the preconditioning oracle (Algorithm 11) and of its LSQR solver
against what Section 6's theorem and the mathematics fix."""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import precondition as P
from paper_2105_11004_amd import workloads as W

D = 60
R_CS = 5 * (D * D + D)   # the CountSketch size of the experiments (eps = 1/2, delta = 1/3)
M = 2 * D                # gamma = 2


def _fig3_matrix(r: float, seed: int, n: int = 10000) -> np.ndarray:
    """The fixed-spectrum matrices of the preconditioning experiment:
    singular values linspace(1, r, 60)."""
    return W.fixed_spectrum(n, np.linspace(1.0, r, D), seed).numpy()


@pytest.mark.parametrize("r", [1e-2, 1e-4, 1e-6, 1e-8, 1e-10])
def test_kappa_of_preconditioned_matrix_meets_the_theorem(r):
    """kappa(A N) <= xi eta (alpha = 0.2, eps = 1/2) whatever kappa(A), for
    the SVD and the pivoted-QR preconditioner alike (N_svd = N_qr U_R with
    U_R orthogonal, so the two kappas agree)."""
    A = _fig3_matrix(r, 11)
    bound = P.kappa_bound(D, M, 0.2, 0.5)
    for seed in range(3):
        Ns, ks = P.count_gauss_precondition(A, seed, R_CS, M, 1e-12, "svd")
        Nq, kq = P.count_gauss_precondition(A, seed, R_CS, M, 1e-12, "qr")
        assert ks == kq == D
        cs, cq = np.linalg.cond(A @ Ns), np.linalg.cond(A @ Nq)
        assert cs <= bound and abs(cs - cq) <= 1e-6 * cs
        assert cs < 20  # far inside the bound, and not growing with kappa(A) = 1 / r


def test_preconditioned_solution_is_the_pseudoinverse_solution():
    """x = N y-hat = A^+ b: full rank, and rank 40 of 60 (the minimum-norm
    solution), against numpy's lstsq."""
    rng = np.random.default_rng(12)
    A = _fig3_matrix(1e-3, 13, n=8000)
    b = rng.standard_normal(A.shape[0])
    N, _ = P.count_gauss_precondition(A, 5, R_CS, M, 1e-12, "svd")
    x, hist = P.preconditioned_lsqr(A, N, b, 80)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert hist[-1] == pytest.approx(np.linalg.norm(A @ xs - b), rel=1e-9)
    # rank 40 of 60: the SVD preconditioner spans range(A^T), so x is the
    # minimum-norm solution; the QR one spans the kept coordinates, so x is a
    # (basic) least-squares solution with the same residual
    B = rng.standard_normal((8000, 40)) @ rng.standard_normal((40, D))
    xs = np.linalg.lstsq(B, b, rcond=1e-10)[0]
    for method in ("svd", "qr"):
        N, k = P.count_gauss_precondition(B, 6, R_CS, M, 1e-8, method)
        assert k == 40
        x, _ = P.preconditioned_lsqr(B, N, b, 80)
        assert np.linalg.norm(B @ x - b) == pytest.approx(np.linalg.norm(B @ xs - b), rel=1e-10)
        if method == "svd":
            assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
        else:
            assert np.count_nonzero(x) == 40


def test_lsqr_matches_the_reference_implementation():
    """The recurrences written out give scipy's LSQR iterates (same start,
    same number of steps, no damping) and converge to the least-squares
    solution."""
    rng = np.random.default_rng(14)
    A = rng.standard_normal((500, 30)) @ np.diag(np.linspace(1, 0.05, 30))
    b = rng.standard_normal(500)
    for it in (1, 5, 20):
        y, _ = P.lsqr(lambda z: A @ z, lambda r: A.T @ r, b, it)
        ref = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=it)[0]
        np.testing.assert_allclose(y, ref, rtol=1e-8, atol=1e-10)
    y, _ = P.lsqr(lambda z: A @ z, lambda r: A.T @ r, b, 200)
    np.testing.assert_allclose(y, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-8)


def test_kappa_bound_formula():
    """xi eta at a few points (the formula of the theorem, by hand)."""
    assert P.kappa_bound(60, 120, 0.2, 0.5) == pytest.approx(
        (1.2 + math.sqrt(0.5)) / (0.8 - math.sqrt(0.5)) * 3.0)
    assert P.kappa_bound(1, 10 ** 8, 0.0, 0.0) == pytest.approx(1.0, abs=1e-3)
