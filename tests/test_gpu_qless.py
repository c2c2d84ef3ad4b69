"""Parity of Algorithm 6 (exact scores from a Q-less column-pivoted QR of A,
lev_params.mode = LEV_MODE_QLESS) through the C-ABI with the FP64 CPU
oracle on the same seeded inputs."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import leverage as L
from paper_2105_11004_amd import api
from paper_2105_11004_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _padded(A: np.ndarray, dtype, device) -> torch.Tensor:
    n, d = A.shape
    es = torch.tensor([], dtype=dtype).element_size()
    ld = -(-d * es // 16) * 16 // es
    buf = torch.zeros(n, ld, dtype=dtype)
    buf[:, :d] = torch.from_numpy(A).to(dtype)
    return buf.to(device)[:, :d]


FORMS = [(torch.float64, "native", 1e-10), (torch.float32, "native", 1e-4), (torch.bfloat16, "bf16x3", 1e-4)]


@pytest.mark.parametrize("form", FORMS, ids=["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("n,d,rank,cap", [(3000 + 7, 12, 12, 12), (20000 + 1, 100, 100, 100), (5000 + 3, 30, 7, 30),
                                          (8000 + 9, 300, 300, 300), (6000 + 5, 520, 520, 40), (4000, 64, 64, 5)])
def test_qless_scores(gpu, form, n, d, rank, cap):
    """Full rank, rank deficient (the cutoff stops the steps), capped steps
    (the scores of the first pivots' columns), and rows of more than 256
    16-byte vectors (FP64 at d = 520)."""
    dtype, prec, bar = form
    if dtype == torch.bfloat16 and rank < d:
        pytest.skip("BF16 rounding of a low-rank product is not low rank")
    _log("qless", dtype, prec, n, d, rank, cap)
    rng = np.random.default_rng(n + d + cap)
    if rank < d:
        A = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, d))
    else:
        A = rng.standard_normal((n, d)) * rng.lognormal(0, 1, (n, 1)) * rng.uniform(0.5, 2.0, d)
    At = _padded(A, dtype, gpu)
    theta = api.lev_estimate(At, 0, 1, 1, cap, 1e-5, precision=prec, mode="qless").cpu().numpy().astype(np.float64)
    ref, q = L.ls_qless_qr(At.cpu().to(torch.float64).numpy(), 1e-5, cap)
    assert q.rank == min(rank, cap)
    rel = _rel(theta, ref)
    _log("qless max rel", rel.max(), "sum", theta.sum(), "rank", q.rank)
    assert rel.max() < bar
    assert abs(theta.sum() - q.rank) < 1e-3 * q.rank


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,d,zero_cols,cap", [(20000 + 3, 64, 8, 64), (50000 + 1, 200, 20, 24)])
def test_qless_scores_csr(gpu, dtype, n, d, zero_cols, cap):
    """CSR input: per step, the rows holding the pivot column are found in a
    sweep over the column ids and only they are read; zero columns are
    never pivots."""
    _log("qless csr", dtype, n, d, zero_cols, cap)
    S = W.sparse_power_law(n, d, zero_cols, n + d).to_scipy()
    S.sort_indices()
    vals = torch.from_numpy(S.data.astype(np.float64)).to(dtype)
    A = api.Csr(torch.from_numpy(S.indptr.astype(np.int64)).to(gpu), torch.from_numpy(S.indices.astype(np.int32)).to(gpu),
                vals.to(gpu), n, d)
    Sh = sp.csr_matrix((vals.to(torch.float64).numpy(), S.indices, S.indptr), shape=(n, d))
    theta = api.lev_estimate(A, 0, 1, 1, cap, 1e-5, mode="qless").cpu().numpy().astype(np.float64)
    ref, q = L.ls_qless_qr(Sh, 1e-5, cap)
    assert q.rank == min(cap, d - zero_cols)
    live = ref > 0
    assert np.all(theta[~live] == 0)
    rel = _rel(theta[live], ref[live])
    bar = 1e-10 if dtype == torch.float64 else 1e-4
    _log("qless csr max rel", rel.max(), "sum", theta.sum())
    assert rel.max() < bar


def test_qless_deterministic_and_empty(gpu):
    """Fixed-order sums: two runs give the same bits (dense and CSR); no rows
    gives rank 0 and no scores."""
    A = torch.from_numpy(np.random.default_rng(5).standard_normal((30000, 48))).float().to(gpu)
    t1 = api.lev_estimate(A, 0, 1, 1, 48, 1e-5, mode="qless")
    t2 = api.lev_estimate(A, 0, 1, 1, 48, 1e-5, mode="qless")
    assert torch.equal(t1, t2)
    S = W.sparse_power_law(40000, 96, 0, 7).to(gpu)
    c1 = api.lev_estimate(S, 0, 1, 1, 96, 1e-5, mode="qless")
    c2 = api.lev_estimate(S, 0, 1, 1, 96, 1e-5, mode="qless")
    assert torch.equal(c1, c2)
    E = torch.zeros(0, 16, dtype=torch.float32, device=gpu)
    assert api.lev_estimate(E, 0, 1, 1, 16, 1e-5, mode="qless").shape == (0,)
