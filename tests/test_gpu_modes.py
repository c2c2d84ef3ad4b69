"""Parity of the wider estimator modes (through the C-ABI) with the FP64 CPU
oracle on the same seeded inputs:

* JL steps with k > 64 columns (pass 2 in column tiles of 64);
* the estimate without the JL step (Pi_2 = I): theta'_i =
  ||e_i^T A_K R11^{-1}||^2, over ceil(r / 64) column tiles;
* Algorithm 7's exact scores for d up to 1024 and on CSR input (the Gram
  route of Algorithm 5: B = A_K^T A_K in one more pass over A);
* the end-to-end (1 +- eps) bound at theory-sized parameters.

Bars: relative per row, 1e-10 for FP64, 1e-4 for the FP32-level forms."""

import math

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


def _csr(S: sp.csr_matrix, dtype, device) -> api.Csr:
    S = S.tocsr()
    S.sort_indices()
    return api.Csr(torch.from_numpy(S.indptr.astype(np.int64)).to(device),
                   torch.from_numpy(S.indices.astype(np.int32)).to(device),
                   torch.from_numpy(S.data.astype(np.float64)).to(dtype).to(device), S.shape[0], S.shape[1])


def _dense(n, d, rank, seed):
    rng = np.random.default_rng(seed)
    if rank < d:
        return rng.standard_normal((n, rank)) @ rng.standard_normal((rank, d))
    return rng.standard_normal((n, d)) * rng.lognormal(0, 1, (n, 1))


def _padded(A: np.ndarray, dtype, device) -> torch.Tensor:
    """Row pitch a multiple of 16 bytes (the interface's requirement)."""
    n, d = A.shape
    es = torch.tensor([], dtype=dtype).element_size()
    ld = -(-d * es // 16) * 16 // es
    buf = torch.zeros(n, ld, dtype=dtype)
    buf[:, :d] = torch.from_numpy(A).to(dtype)
    return buf.to(device)[:, :d]


def _host(At: torch.Tensor) -> np.ndarray:
    return At.cpu().to(torch.float64).numpy()


# (dtype, precision, bar): FP64 MFMA, FP32 storage in BF16x3, BF16 storage
# with Z in three BF16 parts (both FP32-level)
FORMS = [(torch.float64, "native", 1e-10), (torch.float32, "native", 1e-4), (torch.bfloat16, "bf16x3", 1e-4)]


# ------------------------------------------------------------------ k > 64
@pytest.mark.parametrize("form", FORMS, ids=["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("n,d,k", [(5000 + 3, 48, 65), (9000 + 11, 96, 150), (3000, 32, 256)])
def test_jl_column_tiles(gpu, form, n, d, k):
    """Algorithm 10 with k > 64 JL columns: one pass over A per tile of 64
    columns of Z, the squares added into theta (the last tile ragged)."""
    dtype, prec, bar = form
    _log("jl tiles", dtype, prec, n, d, k)
    A = _dense(n, d, d, n + d + k)
    At = _padded(A, dtype, gpu)
    r_cs, m, seed, zeta = 2048, 2 * d, 4040 + k, 1e-5
    theta = api.lev_estimate(At, seed, r_cs, m, k, zeta, precision=prec).cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(_host(At), seed, r_cs, m, k, zeta)
    assert o.rank == d
    rel = _rel(theta, o.theta)
    _log("max rel", rel.max())
    assert rel.max() < bar


def test_jl_column_tiles_csr(gpu):
    n, d, k = 20000 + 7, 200, 130
    S = W.sparse_power_law(n, d, 20, 91).to_scipy()
    A = _csr(S, torch.float32, gpu)
    r_cs, m, seed, zeta = 4096, 2 * d, 515, 1e-5
    theta = api.lev_estimate(A, seed, r_cs, m, k, zeta).cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(S.astype(np.float64), seed, r_cs, m, k, zeta)
    assert o.rank == 180
    live = o.theta > 0
    assert np.all(theta[~live] == 0)
    rel = _rel(theta[live], o.theta[live])
    _log("csr jl tiles max rel", rel.max())
    assert rel.max() < 1e-4


# ------------------------------------------------------------------ no JL step
@pytest.mark.parametrize("form", FORMS, ids=["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("n,d,rank", [(4000 + 1, 40, 40), (6000 + 5, 200, 130), (3000 + 9, 300, 300)])
def test_nojl_estimate(gpu, form, n, d, rank):
    """The estimate without the JL step, theta'_i = ||e_i^T A_K R11^{-1}||^2,
    against the oracle's theta' on its own columns K and R11 (same sketch):
    the same rank and the same column set (theta' depends on the set only)."""
    dtype, prec, bar = form
    if dtype == torch.bfloat16 and rank < d:
        pytest.skip("BF16 rounding of a low-rank product is not low rank")
    _log("nojl", dtype, prec, n, d, rank)
    A = _dense(n, d, rank, 7 * n + d)
    At = _padded(A, dtype, gpu)
    r_cs, m, seed = 4096, 2 * d, 777 + d
    zeta = 1e-10 if dtype == torch.float64 else 1e-5
    theta = api.lev_estimate(At, seed, r_cs, m, 1, zeta, precision=prec, mode="nojl")
    theta = theta.cpu().numpy().astype(np.float64)
    _, st = api.lev_estimate(At, seed, r_cs, m, 8, zeta, precision=prec, return_state=True)
    Ah = _host(At)
    o = L.ls_hrn_approx(Ah, seed, r_cs, m, 8, zeta)
    r = int(st.rank.item())
    assert r == o.rank == rank and int(st.error.item()) == 0
    K = np.sort(o.perm[:r])
    np.testing.assert_array_equal(np.sort(st.perm.cpu().numpy()[:r]), K)
    tp = L.theta_prime(Ah, o.perm[:r], o.R11)
    rel = _rel(theta, tp)
    _log("nojl max rel", rel.max())
    assert rel.max() < bar


def test_nojl_csr_with_zero_columns(gpu):
    n, d = 30000 + 3, 160
    S = W.sparse_power_law(n, d, 16, 92).to_scipy()
    A = _csr(S, torch.float32, gpu)
    r_cs, m, seed, zeta = 4096, 2 * d, 616, 1e-5
    theta = api.lev_estimate(A, seed, r_cs, m, 1, zeta, mode="nojl").cpu().numpy().astype(np.float64)
    Sh = S.astype(np.float64).tocsr()
    o = L.ls_hrn_approx(Sh, seed, r_cs, m, 8, zeta)
    assert o.rank == 144
    tp = L.theta_prime(Sh, o.perm[:o.rank], o.R11)
    live = tp > 0
    assert np.all(theta[~live] == 0)
    rel = _rel(theta[live], tp[live])
    _log("csr nojl max rel", rel.max())
    assert rel.max() < 1e-4


# ------------------------------------------------------------------ exact scores
@pytest.mark.parametrize("form", FORMS, ids=["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("n,d,rank", [(5000 + 7, 100, 100), (8000 + 1, 256, 128), (4000 + 13, 520, 520)])
def test_exact_scores_wide(gpu, form, n, d, rank):
    """Algorithm 7 for d > 64: B = A^T A on the FP64 matrix cores (products
    of FP32 and BF16 values are exact in FP64), the pivoted Cholesky of
    B_K, and pass 2 over the column tiles below the rank, against the
    oracle's Algorithm 7 (eigh of A_K^T A_K)."""
    dtype, prec, bar = form
    if dtype == torch.bfloat16 and rank < d:
        pytest.skip("BF16 rounding of a low-rank product is not low rank")
    _log("exact wide", dtype, prec, n, d, rank)
    A = _dense(n, d, rank, 3 * n + d)
    At = _padded(A, dtype, gpu)
    r_cs, m, seed = 4096, 2 * d, 3131 + d
    zeta = 1e-10 if dtype == torch.float64 else 1e-5
    theta = api.lev_estimate(At, seed, r_cs, m, 1, zeta, precision=prec, mode="exact")
    theta = theta.cpu().numpy().astype(np.float64)
    o = L.ls_hrn_exact(_host(At), seed, r_cs, m, zeta)
    assert o.rank == rank
    rel = _rel(theta, o.theta)
    _log("exact wide max rel", rel.max(), "sum", theta.sum())
    assert rel.max() < bar
    assert abs(theta.sum() - rank) < 1e-3 * rank


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,d,zero_cols", [(20000 + 1, 100, 10), (40000 + 3, 300, 44)])
def test_exact_scores_csr(gpu, dtype, n, d, zero_cols):
    """Algorithm 7 on CSR A: B = A^T A from the rows' nonzero pairs (sum_i
    nnz_i^2 products, FP64 LDS atomics per 128 x 128 tile of B), then the
    same steps as dense; zero columns are left out by the rank."""
    _log("exact csr", dtype, n, d, zero_cols)
    S = W.sparse_power_law(n, d, zero_cols, n + d).to_scipy()
    A = _csr(S, dtype, gpu)
    Sh = sp.csr_matrix((A.values.cpu().to(torch.float64).numpy(), A.col_idx.cpu().numpy(),
                        A.row_ptr.cpu().numpy()), shape=(n, d))
    r_cs, m, seed = 4096, 2 * d, 4242 + d
    zeta = 1e-10 if dtype == torch.float64 else 1e-5
    theta = api.lev_estimate(A, seed, r_cs, m, 1, zeta, mode="exact").cpu().numpy().astype(np.float64)
    o = L.ls_hrn_exact(Sh, seed, r_cs, m, zeta)
    assert o.rank == d - zero_cols
    live = o.theta > 0
    assert np.all(theta[~live] == 0)
    rel = _rel(theta[live], o.theta[live])
    bar = 1e-10 if dtype == torch.float64 else 1e-4
    _log("exact csr max rel", rel.max(), "sum", theta.sum())
    assert rel.max() < bar
    assert abs(theta.sum() - o.rank) < 1e-3 * o.rank


def test_exact_scores_rank_deficient_csr(gpu):
    """Duplicated columns make A_K's Gram singular unless the sketch's
    pivoting drops them: the rank is that of A, the scores the exact ones."""
    n, d = 15000 + 9, 64
    S = W.sparse_power_law(n, d, 0, 93).to_scipy().tolil()
    base = S.tocsc()
    cols = [base[:, j] for j in range(d)]
    cols[40:48] = [cols[j] + cols[j + 1] for j in range(8)]  # 8 dependent columns
    S = sp.hstack(cols).tocsr()
    S.eliminate_zeros()
    A = _csr(S, torch.float64, gpu)
    theta = api.lev_estimate(A, 88, 2048, 2 * d, 1, 1e-10, mode="exact").cpu().numpy()
    o = L.ls_hrn_exact(S.astype(np.float64), 88, 2048, 2 * d, 1e-10)
    assert o.rank == d - 8
    live = o.theta > 0
    rel = _rel(theta[live], o.theta[live])
    _log("exact csr rank-deficient max rel", rel.max())
    assert rel.max() < 1e-9


# ------------------------------------------------------------------ (1 +- eps) end to end
def test_end_to_end_bound_at_theory_sizes(gpu):
    """The composed bound on the GPU: at a CountSketch of at least the OSE
    size (eps = 0.5, delta = 1/3), m = 64 r >= 30 r Gaussian rows and the
    JL bound's k = 400 columns (seven column tiles), every row's theta~_i
    lies within (1 +- 0.5) of the exact theta_i for all but a fraction
    <= delta of the seeds; one seed also against the oracle's theta~."""
    E2E = W.THEORY_SIZED
    A = W.theory_sized_matrix()
    th, _ = L.exact_theta_svd(A, 1e-12)
    At = torch.from_numpy(A).to(gpu)
    seeds, fails = 24, 0
    for seed in range(seeds):
        theta = api.lev_estimate(At, seed, E2E["r_cs"], E2E["m"], E2E["k"], 1e-10).cpu().numpy()
        fails += int(np.max(np.abs(theta / th - 1)) > E2E["eps"])
        if seed == 0:
            o = L.ls_hrn_approx(A, seed, E2E["r_cs"], E2E["m"], E2E["k"], 1e-10)
            assert _rel(theta, o.theta).max() < 1e-10
    _log("e2e fails", fails, "of", seeds)
    assert fails / seeds <= E2E["delta"]


# ------------------------------------------------------------------ full size
def _cfg(name):
    idx = list(W.CONFIGS).index(name) + 1
    return dict(W.CONFIGS[name]), W.data_seed(idx), W.sketch_seed(idx)


def test_exact_scores_full_size_dense_sampled(gpu):
    """Algorithm 7 on the 2^20 x 256 rank-128 FP32 workload (1% of the rows
    scaled by 1e3) in the benchmark's launch configuration: sampled rows
    against the oracle's Algorithm 7 run on the whole matrix."""
    cfg, dseed, seed = _cfg("dense_f32_1Mx256_rank128")
    n, d = cfg["n"], cfg["d"]
    A = W.low_rank_coherent(n, d, cfg["rank"], dseed, device=gpu)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], mode="exact")
    theta = plan.run().cpu().numpy().astype(np.float64)
    rows = np.sort(np.random.default_rng(61).choice(n, 3000, replace=False))
    o = L.ls_hrn_exact(A.cpu().numpy().astype(np.float64), seed, cfg["r_cs"], cfg["m"], cfg["zeta"], rows=rows)
    assert o.rank == cfg["rank"]
    rel = _rel(theta[rows], o.theta_rows)
    _log("exact dense full size max rel", rel.max(), "sum", theta.sum())
    assert rel.max() < 1e-4 and abs(theta.sum() - o.rank) < 1e-3 * o.rank


def test_exact_scores_full_size_csr_sampled(gpu):
    """Algorithm 7 on the 2^23 x 512 CSR workload (64 zero columns): the
    sketch keeps the 448 live columns, so the exact scores of A_K are those
    of A; sampled rows against the oracle's exact scores of A (the Gram of A
    streamed over row blocks, Algorithm 5), and sum theta = 448."""
    cfg, dseed, seed = _cfg("csr_f32_8Mx512")
    n, d = cfg["n"], cfg["d"]
    A = W.sparse_power_law(n, d, cfg["zero_cols"], dseed, device=gpu)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], mode="exact")
    theta = plan.run().cpu().numpy().astype(np.float64)
    live_rank = d - cfg["zero_cols"]
    _log("exact csr full size sum", theta.sum())
    assert abs(theta.sum() - live_rank) < 1e-3 * live_rank
    S = A.to_scipy()
    rows = np.sort(np.random.default_rng(62).choice(n, 3000, replace=False))
    blk = 1 << 18
    chunks = lambda: ((lo, S[lo:lo + blk].toarray()) for lo in range(0, n, blk))  # noqa: E731
    exact, rho = L.theta_gram_rows(chunks, rows, 1e-6)
    assert rho == live_rank
    live = exact > 0
    assert np.all(theta[rows][~live] == 0)
    rel = _rel(theta[rows][live], exact[live])
    _log("exact csr full size max rel", rel.max())
    assert rel.max() < 1e-4
