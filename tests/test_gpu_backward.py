"""The adjoint kernels (lev_estimate_backward, through the C-ABI and the
autograd Function) against the FP64 reference gradient of the oracle, and
against finite differences of the GPU's own FP64 forward."""

import numpy as np
import pytest
import torch

from oracle import gradient as Gr
from paper_2105_11004_amd import api
from paper_2105_11004_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _weights(n, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.rand(n, generator=g, dtype=torch.float64)


def _compare(gpu_grad, ref_grad, bar):
    """Error per entry relative to the largest gradient entry of its row
    (rows carry very different scales); returns the worst row."""
    err = np.abs(gpu_grad - ref_grad).max(axis=1)
    scale = np.abs(ref_grad).max(axis=1)
    live = scale > 0
    assert np.all(err[~live] == 0)
    rel = err[live] / scale[live]
    _log("grad max row-rel err", rel.max(), "p99", np.quantile(rel, 0.99))
    assert rel.max() < bar
    return rel.max()


@pytest.mark.parametrize("dtype,n,d,k,r_cs,m,bar", [
    (torch.float64, 4096 + 5, 64, 32, 1024, 256, 1e-9),
    (torch.float32, 8192 + 3, 48, 16, 512, 96, 1e-5),
    (torch.float32, 5000 + 7, 80, 64, 1024, 160, 1e-5),
    (torch.float64, 1000, 20, 7, 100, 40, 1e-9),
    # the register-resident FP32 passes with one, two and three 16-column
    # blocks of Z_full
    (torch.float32, 4096 + 9, 64, 16, 1024, 128, 1e-5),
    (torch.float32, 3000 + 1, 96, 32, 1024, 192, 1e-5),
    (torch.float32, 6000 + 11, 128, 40, 2048, 256, 1e-5),
])
def test_backward_matches_reference_gradient(gpu, dtype, n, d, k, r_cs, m, bar):
    _log("bwd", dtype, n, d, k)
    A = W.dense_gaussian(n, d, 31 + d, dtype=dtype)
    w = _weights(n, 5)
    zeta = 1e-10 if dtype == torch.float64 else 1e-5
    Ad = A.to(gpu)
    theta, st = api.lev_estimate(Ad, 7, r_cs, m, k, zeta, return_state=True)
    g = api.lev_estimate_backward(Ad, st, w.to(dtype).to(gpu), 7, r_cs, m, k, zeta).cpu().numpy()
    ref = Gr.estimate_and_gradient(A.to(torch.float64).numpy(), 7, r_cs, m, k, zeta,
                                   w.to(dtype).to(torch.float64).numpy())
    assert int(st.rank.item()) == ref.rank
    np.testing.assert_array_equal(st.perm.cpu().numpy()[:ref.rank], ref.perm[:ref.rank])
    _compare(g.astype(np.float64), ref.grad, bar)


def test_backward_rank_deficient_workload_shape(gpu):
    """The backward workload's shape (256 columns of rank 192, w ~ U(0,1)) at
    2^16 + 3 rows: zero gradient on the 64 unselected columns."""
    n, d, rank, r_cs, m, k, zeta = 65536 + 3, 256, 192, 4096, 512, 48, 1e-5
    A = W.low_rank_coherent(n, d, rank, 1005, heavy_frac=0.0)
    w = _weights(n, 6).to(torch.float32)
    Ad = A.to(gpu)
    theta, st = api.lev_estimate(Ad, 2005, r_cs, m, k, zeta, return_state=True)
    g = api.lev_estimate_backward(Ad, st, w.to(gpu), 2005, r_cs, m, k, zeta).cpu().numpy()
    ref = Gr.estimate_and_gradient(A.numpy().astype(np.float64), 2005, r_cs, m, k, zeta,
                                   w.numpy().astype(np.float64))
    r = int(st.rank.item())
    assert r == ref.rank == rank
    notK = st.perm.cpu().numpy()[r:]
    assert np.all(g[:, notK] == 0)
    _compare(g.astype(np.float64), ref.grad, 1e-5)
    # <grad, A> = 0 (theta~ is scale invariant at a fixed sketch)
    ip = float(np.sum(g.astype(np.float64) * A.numpy()))
    assert abs(ip) <= 1e-3 * np.linalg.norm(g) * np.linalg.norm(A.numpy())


def test_backward_full_size_sampled(gpu):
    """The backward workload at full size (2^20 x 256 FP32, rank 192) in the
    launch configuration of the benchmark, checked on sampled rows."""
    cfg = W.CONFIGS["dense_f32_1Mx256_rank192_bwd"]
    n, d = cfg["n"], cfg["d"]
    _log("bwd full size: generating")
    A = W.low_rank_coherent(n, d, cfg["rank"], W.data_seed(5), heavy_frac=0.0, device=gpu)
    w = torch.rand(n, generator=torch.Generator(device=gpu).manual_seed(5), device=gpu, dtype=torch.float32)
    theta, st = api.lev_estimate(A, W.sketch_seed(5), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"],
                                 return_state=True)
    g = api.lev_estimate_backward(A, st, w, W.sketch_seed(5), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"])
    assert torch.all(torch.isfinite(g))
    rows = np.sort(np.random.default_rng(3).choice(n, 2000, replace=False))
    g_rows = g[torch.from_numpy(rows).to(gpu)].cpu().numpy().astype(np.float64)
    _log("bwd full size: oracle")
    ref = Gr.estimate_and_gradient(A.cpu().numpy().astype(np.float64), W.sketch_seed(5), cfg["r_cs"], cfg["m"],
                                   cfg["k"], cfg["zeta"], w.cpu().numpy().astype(np.float64))
    assert ref.rank == cfg["rank"]
    _compare(g_rows, ref.grad[rows], 1e-5)


def test_backward_finite_differences_on_a_slice(gpu):
    """The 2048 x 32 slice as a standalone FP64 problem: directional
    derivatives of the GPU forward (central differences, pivots unchanged by
    the step) against <grad, E> of the GPU backward."""
    A = W.low_rank_coherent(2048, 32, 32, 77, heavy_frac=0.0, dtype=torch.float64).to(gpu)
    w = _weights(2048, 8).to(gpu)
    r_cs, m, k, zeta, seed = 512, 64, 16, 1e-10, 11
    theta, st = api.lev_estimate(A, seed, r_cs, m, k, zeta, return_state=True)
    g = api.lev_estimate_backward(A, st, w, seed, r_cs, m, k, zeta)
    perm0 = st.perm.clone()
    gen = torch.Generator(device=gpu).manual_seed(4)
    f0 = float(w @ theta)
    # Central differences are exact to O(h^2 |E|^2) up to the forward's
    # rounding, which the factorisation through the Gram matrix A~^T A~
    # scales by kappa(A~)^2 (kappa from R's diagonal): allow
    # |fd - an| <= 1e-6 |an| + 64 eps kappa^2 |f| / h.  Dense random
    # directions (|E| ~ 256) take h = 1e-6, single entries h = 1e-4.
    r = int(st.rank.item())
    dg = torch.diagonal(st.R)[:r]
    kappa = float(dg[0] / dg[r - 1])
    _log("kappa", kappa)
    worst = 0.0
    for trial in range(12):
        E = torch.randn(A.shape, generator=gen, device=gpu, dtype=torch.float64)
        h = 1e-6
        if trial >= 8:  # single entries
            E = torch.zeros_like(A)
            E[(trial * 523) % 2048, (trial * 7) % 32] = 1.0
            h = 1e-4
        noise = 64 * np.finfo(np.float64).eps * kappa ** 2 * abs(f0) / h
        tp, sp = api.lev_estimate(A + h * E, seed, r_cs, m, k, zeta, return_state=True)
        tm, sm = api.lev_estimate(A - h * E, seed, r_cs, m, k, zeta, return_state=True)
        assert torch.equal(sp.perm, perm0) and torch.equal(sm.perm, perm0)
        fd = float((w @ tp - w @ tm) / (2 * h))
        an = float(torch.sum(g * E))
        _log("trial", trial, "fd", fd, "grad", an, "diff", fd - an, "allowed", 1e-6 * abs(an) + noise)
        worst = max(worst, abs(fd - an) / (1e-6 * abs(an) + noise))
    assert worst < 1.0


def test_autograd_function(gpu):
    A = W.dense_gaussian(3000, 24, 9, dtype=torch.float32).to(gpu).requires_grad_(True)
    theta = api.estimate(A, 3, 256, 64, 8, 1e-5)
    w = torch.rand(3000, device=gpu)
    (gA,) = torch.autograd.grad(theta, A, grad_outputs=w)
    _, st = api.lev_estimate(A.detach(), 3, 256, 64, 8, 1e-5, return_state=True)
    g2 = api.lev_estimate_backward(A.detach(), st, w, 3, 256, 64, 8, 1e-5)
    assert torch.equal(gA, g2)
    # the loss's gradient through a weighted sum
    loss = (theta.detach() * 0 + api.estimate(A, 3, 256, 64, 8, 1e-5)).sum()
    loss.backward()
    assert A.grad is not None and torch.all(torch.isfinite(A.grad))
