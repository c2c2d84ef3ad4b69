"""Pins of the reference gradient (oracle.gradient) to things other than
itself: central finite differences of the oracle's forward estimator, an
independent reverse-mode route (torch autograd in FP64 on the CPU, through
torch.linalg.qr), and invariants of the estimator."""

import numpy as np
import pytest
import torch

from oracle import conventions as C
from oracle import gradient as Gr
from oracle import leverage as L


def _problem(n=48, d=7, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, d)) * rng.uniform(0.3, 3.0, size=(n, 1))
    w = rng.uniform(0.0, 1.0, n)
    return A, w


PARAMS = dict(seed=17, r_cs=24, m=14, k_jl=5, zeta=1e-10)


def _f(A, w, perm, rank):
    """f = w^T theta~ from the oracle's forward estimator with the pivots
    held fixed (its QRCP replaced by the given perm and rank)."""
    n, d = A.shape
    rnd = C.derive(PARAMS["seed"], n, PARAMS["r_cs"])
    At = C.gaussian_transform(rnd, PARAMS["m"]) @ L.countsketch_apply(rnd, A)
    K = perm[:rank]
    R = L.r_from_qr_of_sketch(At[:, K])
    Z = L.jl_orthogonalizer(R, C.jl_gaussian(rnd, d, PARAMS["k_jl"])[:rank])
    return float(w @ L.row_norms_sq(A[:, K], Z))


def test_gradient_matches_central_differences():
    A, w = _problem()
    g = Gr.estimate_and_gradient(A, w=w, **PARAMS)
    assert g.rank == A.shape[1]
    assert abs(g.f - _f(A, w, g.perm, g.rank)) <= 1e-12 * abs(g.f)
    h = 1e-5
    fd = np.empty_like(A)
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            E = np.zeros_like(A)
            E[i, j] = h
            fd[i, j] = (_f(A + E, w, g.perm, g.rank) - _f(A - E, w, g.perm, g.rank)) / (2 * h)
    scale = np.abs(g.grad).max()
    assert np.abs(fd - g.grad).max() <= 1e-7 * scale


def test_gradient_rank_deficient_matches_central_differences():
    """r < d: the unselected columns get exactly zero gradient, the selected
    ones match finite differences."""
    rng = np.random.default_rng(5)
    n, d = 60, 8
    A = rng.standard_normal((n, 5)) @ rng.standard_normal((5, d))
    w = rng.uniform(0, 1, n)
    g = Gr.estimate_and_gradient(A, w=w, **{**PARAMS, "zeta": 1e-8})
    assert g.rank == 5
    notK = g.perm[g.rank:]
    assert np.all(g.grad[:, notK] == 0)
    h = 1e-6
    for i in (0, 17, 59):
        for j in g.perm[:g.rank]:
            E = np.zeros_like(A)
            E[i, j] = h
            fd = (_f(A + E, w, g.perm, g.rank) - _f(A - E, w, g.perm, g.rank)) / (2 * h)
            assert abs(fd - g.grad[i, j]) <= 1e-6 * np.abs(g.grad).max()


def test_gradient_matches_torch_autograd():
    """Independent route: the forward written with torch ops on the dense
    S and G of the same seed, differentiated by torch (its QR backward)."""
    A, w = _problem(n=64, d=9, seed=3)
    g = Gr.estimate_and_gradient(A, w=w, **PARAMS)
    n, d = A.shape
    rnd = C.derive(PARAMS["seed"], n, PARAMS["r_cs"])
    S = torch.from_numpy(L.countsketch_dense_S(rnd))
    G = torch.from_numpy(C.gaussian_transform(rnd, PARAMS["m"]))
    Pi2 = torch.from_numpy(C.jl_gaussian(rnd, d, PARAMS["k_jl"])[:g.rank])
    K = torch.from_numpy(g.perm[:g.rank])
    At = torch.tensor(A, requires_grad=True)
    Q, R = torch.linalg.qr((G @ (S @ At))[:, K])
    R = R * torch.sign(torch.diagonal(R))[:, None]
    Z = torch.linalg.solve_triangular(R, Pi2, upper=True)
    f = (torch.from_numpy(w) * ((At[:, K] @ Z) ** 2).sum(1)).sum()
    f.backward()
    assert abs(f.item() - g.f) <= 1e-12 * abs(g.f)
    np.testing.assert_allclose(At.grad.numpy(), g.grad, rtol=0, atol=1e-10 * np.abs(g.grad).max())


def test_countsketch_transpose_is_the_adjoint():
    """<S A, X> = <A, S^T X> for the dense S of the same seed."""
    rng = np.random.default_rng(2)
    rnd = C.derive(8, 50, 12)
    A, X = rng.standard_normal((50, 3)), rng.standard_normal((12, 3))
    S = L.countsketch_dense_S(rnd)
    np.testing.assert_allclose(Gr.countsketch_transpose_apply(rnd, X), S.T @ X, rtol=1e-15)
    assert abs(np.sum(L.countsketch_apply(rnd, A) * X) - np.sum(A * Gr.countsketch_transpose_apply(rnd, X))) < 1e-12


def test_gradient_invariants():
    A, w = _problem(n=80, d=6, seed=9)
    g = Gr.estimate_and_gradient(A, w=w, **PARAMS)
    # theta~(cA) = theta~(A) at a fixed sketch (R scales by c, Z by 1/c), so
    # the gradient is orthogonal to A
    assert abs(np.sum(g.grad * A)) <= 1e-12 * np.linalg.norm(g.grad) * np.linalg.norm(A)
    # linear in w
    g2 = Gr.estimate_and_gradient(A, w=3.0 * w, **PARAMS)
    np.testing.assert_allclose(g2.grad, 3.0 * g.grad, rtol=1e-12, atol=1e-15)
    # theta~ and f agree with the forward estimator
    est = L.ls_hrn_approx(A, PARAMS["seed"], PARAMS["r_cs"], PARAMS["m"], PARAMS["k_jl"], PARAMS["zeta"])
    np.testing.assert_allclose(g.theta, est.theta, rtol=1e-12)
    # zero weights give a zero gradient
    assert np.all(Gr.estimate_and_gradient(A, w=0 * w, **PARAMS).grad == 0)


def _fd_error(grad_fn):
    A, w = _problem(n=30, d=5, seed=11)
    g = grad_fn(A, w)
    h = 1e-5
    fd = np.empty_like(A)
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            E = np.zeros_like(A)
            E[i, j] = h
            fd[i, j] = (_f(A + E, w, g.perm, g.rank) - _f(A - E, w, g.perm, g.rank)) / (2 * h)
    return np.abs(fd - g.grad).max() / np.abs(g.grad).max()


def test_pins_catch_a_wrong_qr_adjoint(monkeypatch):
    good = _fd_error(lambda A, w: Gr.estimate_and_gradient(A, w=w, **PARAMS))
    monkeypatch.setattr(Gr, "copyltu", lambda M: np.tril(M))
    bad = _fd_error(lambda A, w: Gr.estimate_and_gradient(A, w=w, **PARAMS))
    assert good < 1e-7 and bad > 1e-3


def test_pins_catch_a_flipped_sketch_sign(monkeypatch):
    good = Gr.countsketch_transpose_apply
    monkeypatch.setattr(Gr, "countsketch_transpose_apply", lambda rnd, X: -good(rnd, X))
    bad = _fd_error(lambda A, w: Gr.estimate_and_gradient(A, w=w, **PARAMS))
    assert bad > 1e-3
