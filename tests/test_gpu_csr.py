"""Parity of the CSR path (pass 1 and pass 2 on sparse A, through the C-ABI)
with the FP64 CPU oracle on the same seeded inputs."""

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


def _csr_from_scipy(S: sp.csr_matrix, dtype, device) -> api.Csr:
    S = S.tocsr()
    S.sort_indices()
    return api.Csr(torch.from_numpy(S.indptr.astype(np.int64)).to(device),
                   torch.from_numpy(S.indices.astype(np.int32)).to(device),
                   torch.from_numpy(S.data.astype(np.float64)).to(dtype).to(device), S.shape[0], S.shape[1])


def _host_f64(A: api.Csr) -> sp.csr_matrix:
    return sp.csr_matrix((A.values.cpu().to(torch.float64).numpy(), A.col_idx.cpu().numpy(),
                          A.row_ptr.cpu().numpy()), shape=(A.n, A.d))


def _ragged_csr(n, d, seed, long_rows=(), empty_rows=(), integer=False):
    """Power-law rows plus planted rows of given lengths (and empty rows)."""
    rng = np.random.default_rng(seed)
    A = W.sparse_power_law(n, d, max(1, d // 8), seed).to_scipy().tolil()
    for i, ell in long_rows:
        cols = np.sort(rng.choice(d, size=ell, replace=False))
        A.rows[i] = list(cols)
        A.data[i] = list(rng.standard_normal(ell))
    for i in empty_rows:
        A.rows[i] = []
        A.data[i] = []
    A = A.tocsr()
    if integer:
        A.data = np.round(A.data * 4.0)
        A.eliminate_zeros()
    return A


# ------------------------------------------------------------------ pass 1
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.bfloat16])
def test_csr_sketch_integer_values_bit_exact(gpu, dtype):
    """Integer-valued A: every FP64 partial sum is exact, so S A is the same
    bits in any accumulation order."""
    n, d, r_cs, m = 20011, 512, 1024, 512
    _log("csr sketch", dtype)
    S = _ragged_csr(n, d, 3, long_rows=[(5, 448), (6, 65), (7, 64), (8, 129), (n - 1, 300)],
                    empty_rows=[0, 100, n - 2], integer=True)
    A = _csr_from_scipy(S, dtype, gpu)
    At, SA = api.lev_sketch(A, 41, r_cs, m, return_sa=True)
    rnd = C.derive(41, n, r_cs)
    SA_o = L.countsketch_apply(rnd, S)
    np.testing.assert_array_equal(SA.cpu().numpy(), SA_o)
    G = C.gaussian_transform(rnd, m)
    At_o = G @ SA_o
    bound = 1e-13 * (np.abs(G) @ np.abs(SA_o)) + 1e-300
    assert np.all(np.abs(At.cpu().numpy() - At_o) <= bound)


def test_csr_sketch_matches_dense_sketch_and_is_deterministic(gpu):
    """The CSR and dense pass-1 kernels accumulate the same FP64 sums (the
    same rows in the same bucket order), and repeated runs agree bitwise."""
    n, d = 30011, 200
    S = W.sparse_power_law(n, d, 8, 12).to_scipy()
    A = _csr_from_scipy(S, torch.float32, gpu)
    D = torch.from_numpy(S.toarray().astype(np.float32)).to(gpu)
    a1, s1 = api.lev_sketch(A, 5, 512, 256, return_sa=True)
    a2, s2 = api.lev_sketch(A, 5, 512, 256, return_sa=True)
    assert torch.equal(s1, s2) and torch.equal(a1, a2)
    _, sd = api.lev_sketch(D, 5, 512, 256, return_sa=True)
    rnd = C.derive(5, n, 512)
    SA_o = L.countsketch_apply(rnd, S)
    scale = np.abs(SA_o).max()
    assert np.abs(s1.cpu().numpy() - SA_o).max() <= 1e-12 * scale
    assert np.abs(sd.cpu().numpy() - SA_o).max() <= 1e-12 * scale


# ------------------------------------------------------------------ the estimator on CSR
def test_csr_estimate_fp32_rank_from_zero_columns(gpu):
    """The sparse workload's shape at 2^16 + 7 rows: 512 columns, 64 of them
    all-zero, so the revealed rank is exactly 448."""
    n, d, nz, r_cs, m, k, zeta, seed = 65536 + 7, 512, 64, 8192, 1024, 64, 1e-5, 2003
    Ah = W.sparse_power_law(n, d, nz, W.data_seed(3))
    A = Ah.to(gpu)
    theta, st = api.lev_estimate(A, seed, r_cs, m, k, zeta, return_state=True)
    S = Ah.to_scipy()
    o = L.ls_hrn_approx(S, seed, r_cs, m, k, zeta)
    r = int(st.rank.item())
    assert r == o.rank == d - nz
    np.testing.assert_array_equal(st.perm.cpu().numpy()[:r], o.perm[:r])
    assert set(st.perm.cpu().numpy()[r:].tolist()) == set(Ah.zero_cols.tolist())
    rel = _rel(theta.cpu().numpy().astype(np.float64), o.theta)
    _log("csr fp32 max rel", rel.max(), "p99", np.quantile(rel, 0.99))
    assert rel.max() < 1e-4


@pytest.mark.parametrize("dtype,d,k,bar", [(torch.float64, 128, 32, 1e-9), (torch.float64, 512, 48, 1e-9),
                                           (torch.float32, 1024, 64, 1e-4), (torch.bfloat16, 256, 16, 1e-4),
                                           (torch.float32, 40, 5, 1e-4)])
def test_csr_estimate_dtypes_and_z_placement(gpu, dtype, d, k, bar):
    """FP64 values take the FP64 path; FP32/BF16 values the FP32 path.  Z_full
    sits in LDS when d * 64 elements fit (d=128 FP64, d=256 and 40 FP32) and
    is read from global memory otherwise (d=512 FP64, d=1024 FP32)."""
    n, r_cs, m, zeta, seed = 20000 + 3, 2048, max(2 * d, 64), 1e-5 if dtype != torch.float64 else 1e-10, 77
    _log("csr", dtype, d, k)
    S = W.sparse_power_law(n, d, d // 8, d + k, mean_nnz=min(16.0, d / 4)).to_scipy()
    A = _csr_from_scipy(S, dtype, gpu)
    theta, st = api.lev_estimate(A, seed, r_cs, m, k, zeta, return_state=True)
    Sh = _host_f64(A)  # the stored values (BF16-rounded where A is BF16)
    o = L.ls_hrn_approx(Sh, seed, r_cs, m, k, zeta)
    r = int(st.rank.item())
    assert r == o.rank
    np.testing.assert_array_equal(st.perm.cpu().numpy()[:r], o.perm[:r])
    rel = _rel(theta.cpu().numpy().astype(np.float64), o.theta)
    _log("max rel", rel.max())
    assert rel.max() < bar


def test_csr_long_empty_and_boundary_rows(gpu):
    """Rows longer than one 64-entry staging chunk, rows that straddle the
    chunks and the 64-row tasks, empty rows at task starts and ends."""
    n, d, r_cs, m, k, zeta = 4096 + 11, 448, 512, 512, 32, 1e-5
    long_rows = [(63, 448), (64, 447), (127, 200), (128, 65), (129, 64), (130, 63), (n - 1, 448)]
    empty = [0, 1, 62, 191, 192, 4095, n - 2]
    S = _ragged_csr(n, d, 21, long_rows=long_rows, empty_rows=empty)
    A = _csr_from_scipy(S, torch.float32, gpu)
    theta = api.lev_estimate(A, 3, r_cs, m, k, zeta).cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(_host_f64(A), 3, r_cs, m, k, zeta)
    assert np.all(theta[empty] == 0)
    keep = np.setdiff1d(np.arange(n), empty)
    rel = _rel(theta[keep], o.theta[keep])
    _log("boundary rows max rel", rel.max())
    assert rel.max() < 1e-4


def test_csr_degenerate(gpu):
    # no nonzeros at all: rank 0, theta = 0
    n, d = 1000, 64
    A = api.Csr(torch.zeros(n + 1, dtype=torch.int64, device=gpu), torch.zeros(0, dtype=torch.int32, device=gpu),
                torch.zeros(0, dtype=torch.float32, device=gpu), n, d)
    theta, st = api.lev_estimate(A, 1, 64, 64, 8, 1e-5, return_state=True)
    assert int(st.rank.item()) == 0 and torch.all(theta == 0)
    # one row, one nonzero
    A = api.Csr(torch.tensor([0, 1], dtype=torch.int64, device=gpu), torch.tensor([3], dtype=torch.int32, device=gpu),
                torch.tensor([2.5], dtype=torch.float32, device=gpu), 1, 8)
    theta = api.lev_estimate(A, 1, 4, 8, 4, 1e-5).cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(_host_f64(A), 1, 4, 8, 4, 1e-5)
    assert _rel(theta, o.theta).max() < 1e-4
    # torch's own CSR layout
    S = W.sparse_power_law(3000, 96, 4, 5).to_scipy()
    T = torch.sparse_csr_tensor(torch.from_numpy(S.indptr.astype(np.int64)),
                                torch.from_numpy(S.indices.astype(np.int64)),
                                torch.from_numpy(S.data.astype(np.float32)), size=S.shape).to(gpu)
    theta = api.lev_estimate(T, 2, 256, 192, 8, 1e-5).cpu().numpy().astype(np.float64)
    o = L.ls_hrn_approx(S, 2, 256, 192, 8, 1e-5)
    assert _rel(theta, o.theta).max() < 1e-4


def test_csr_full_size_sampled(gpu):
    """The sparse workload at full size (2^23 x 512 CSR FP32, 64 zero
    columns, mean 16 nonzeros per row) in the launch configuration the
    benchmark uses, checked on sampled rows against the oracle run on the
    whole matrix."""
    cfg = W.CONFIGS["csr_f32_8Mx512"]
    _log("csr full size: generating")
    A = W.sparse_power_law(cfg["n"], cfg["d"], cfg["zero_cols"], W.data_seed(3), device=gpu)
    plan = api.EstimatePlan(A, W.sketch_seed(3), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"])
    theta = plan.run().cpu().numpy().astype(np.float64)
    assert np.all(theta >= 0) and np.all(np.isfinite(theta))
    _log("csr full size: oracle")
    S = A.to_scipy()
    rows = np.sort(np.random.default_rng(1).choice(cfg["n"], 3000, replace=False))
    o = L.ls_hrn_approx(S, W.sketch_seed(3), cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], rows=rows)
    assert o.rank == cfg["d"] - cfg["zero_cols"]
    rel = _rel(theta[rows], o.theta_rows)
    _log("csr full size max rel", rel.max())
    assert rel.max() < 1e-4
