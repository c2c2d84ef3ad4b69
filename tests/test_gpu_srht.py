"""Parity of the SRHT sketch (A~ = F (S A), the F S composition of Section 4)
through the C-ABI with the FP64 CPU oracle on the same seeded inputs."""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import conventions as C
from oracle import leverage as L
from paper_2105_11004_amd import api
from paper_2105_11004_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _padded(A: np.ndarray, device) -> torch.Tensor:
    """FP64 rows padded to a 16-byte pitch (the interface's requirement)."""
    n, d = A.shape
    buf = torch.zeros(n, d + (d % 2), dtype=torch.float64)
    buf[:, :d] = torch.from_numpy(A)
    return buf.to(device)[:, :d]


@pytest.mark.parametrize("n,d,r_cs,m", [(100, 1, 1, 1), (300, 2, 2, 2), (2000, 33, 64, 40), (5000, 20, 128, 128),
                                        (20000, 100, 1024, 200), (70000, 40, 16384, 96), (50000, 9, 8192, 8192)])
def test_srht_of_the_sketch(gpu, n, d, r_cs, m):
    """F (S A) on the GPU against the oracle's SRHT applied to the GPU's own
    S A: radix passes of 2^8 (one, or two at r_cs = 2^13, 2^14), the signs,
    the sampled rows and the 1 / sqrt(m) scale.  H only adds and subtracts,
    so the error is a few ulps of the largest partial sums."""
    _log("srht", n, d, r_cs, m)
    A = _padded(np.random.default_rng(n + d).standard_normal((n, d)), gpu)
    At, SA = api.lev_sketch(A, 77 + r_cs, r_cs, m, return_sa=True, sketch="srht")
    SAh = SA.cpu().numpy()
    ref = L.srht_apply(C.derive(77 + r_cs, n, r_cs), SAh, m)
    scale = np.abs(SAh).sum(axis=0).max() / math.sqrt(m)
    err = np.abs(At.cpu().numpy() - ref).max()
    _log("srht max abs err", err, "scale", scale)
    assert err <= 1e-14 * max(1.0, math.log2(r_cs)) * scale


FORMS = [(torch.float64, "native", 1e-10), (torch.float32, "native", 1e-4), (torch.bfloat16, "bf16x3", 1e-4)]


@pytest.mark.parametrize("form", FORMS, ids=["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("n,d,r_cs,m,k", [(6000 + 1, 24, 1024, 96, 16), (20000 + 3, 128, 4096, 256, 48)])
def test_srht_estimate(gpu, form, n, d, r_cs, m, k):
    """Algorithm 10 with Pi_1 = F S against the oracle's (same sketch, same
    steps): rank, pivots, theta~."""
    dtype, prec, bar = form
    _log("srht estimate", dtype, prec, n, d)
    rng = np.random.default_rng(n + 3 * d)
    A = rng.standard_normal((n, d)) * rng.lognormal(0, 1, (n, 1))
    At = torch.from_numpy(A).to(dtype).to(gpu)
    zeta = 1e-10 if dtype == torch.float64 else 1e-5
    theta = api.lev_estimate(At, 1234, r_cs, m, k, zeta, precision=prec, sketch="srht")
    o = L.ls_hrn_approx(At.cpu().to(torch.float64).numpy(), 1234, r_cs, m, k, zeta, sketch="srht")
    assert o.rank == d
    rel = _rel(theta.cpu().numpy().astype(np.float64), o.theta)
    _log("srht estimate max rel", rel.max())
    assert rel.max() < bar


def test_srht_estimate_csr_and_exact(gpu):
    """The SRHT sketch on CSR input (zero columns left out by the rank), for
    the JL estimate and for Algorithm 7's exact scores."""
    n, d = 30000 + 7, 96
    S = W.sparse_power_law(n, d, 12, 95).to_scipy()
    S.sort_indices()
    A = api.Csr(torch.from_numpy(S.indptr.astype(np.int64)).to(gpu), torch.from_numpy(S.indices.astype(np.int32)).to(gpu),
                torch.from_numpy(S.data.astype(np.float32)).to(gpu), n, d)
    Sh = sp.csr_matrix((S.data.astype(np.float32).astype(np.float64), S.indices, S.indptr), shape=(n, d))
    theta = api.lev_estimate(A, 55, 2048, 2 * d, 32, 1e-5, sketch="srht").cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(Sh, 55, 2048, 2 * d, 32, 1e-5, sketch="srht")
    assert o.rank == d - 12
    live = o.theta > 0
    assert np.all(theta[~live] == 0)
    rel = _rel(theta[live], o.theta[live])
    _log("srht csr max rel", rel.max())
    assert rel.max() < 1e-4
    ex = api.lev_estimate(A, 55, 2048, 2 * d, 1, 1e-5, mode="exact", sketch="srht").cpu().numpy()
    oe = L.ls_hrn_exact(Sh, 55, 2048, 2 * d, 1e-5, sketch="srht")
    rel = _rel(ex[live].astype(np.float64), oe.theta[live])
    _log("srht csr exact max rel", rel.max())
    assert rel.max() < 1e-4


def test_srht_full_size_bf16_sampled(gpu):
    """The 2^22 x 1024 BF16 workload with the SRHT in place of the Gaussian
    stage (r_cs = 2^14, m = 2048), in the FP32-level form, on sampled rows
    against the oracle's same-sketch estimate."""
    name = "dense_bf16_4Mx1024"
    idx = list(W.CONFIGS).index(name) + 1
    cfg = W.CONFIGS[name]
    A = W.row_scaled_bf16(cfg["n"], cfg["d"], W.data_seed(idx), device=gpu)
    plan = api.EstimatePlan(A, W.sketch_seed(idx), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"],
                            precision="bf16x3", sketch="srht")
    theta = plan.run().cpu().numpy().astype(np.float64)
    rows = np.sort(np.random.default_rng(63).choice(cfg["n"], 2000, replace=False))
    o = L.ls_hrn_approx(A.float().cpu().numpy(), W.sketch_seed(idx), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"],
                        rows=rows, sketch="srht")
    assert o.rank == cfg["d"]
    rel = _rel(theta[rows], o.theta_rows)
    _log("srht full size max rel", rel.max(), "p99", np.quantile(rel, 0.99))
    assert rel.max() < 1e-4
