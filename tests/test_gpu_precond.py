"""Parity of Section 6's preconditioner (Algorithm 11) and LSQR on A N
through the C-ABI with the FP64 CPU oracle on the same seeded inputs."""

import numpy as np
import pytest
import torch

from oracle import precondition as P
from paper_2105_11004_amd import api
from paper_2105_11004_amd import workloads as W

pytestmark = pytest.mark.gpu

D = 60
R_CS = 5 * (D * D + D)
M = 2 * D


def _log(*a):
    print(*a, flush=True)


def _padded(A: np.ndarray, dtype, device) -> torch.Tensor:
    """Rows padded to a 16-byte pitch (the interface's requirement)."""
    n, d = A.shape
    es = torch.tensor([], dtype=dtype).element_size()
    ld = -(-d * es // 16) * 16 // es
    buf = torch.zeros(n, ld, dtype=dtype)
    buf[:, :d] = torch.from_numpy(A).to(dtype)
    return buf.to(device)[:, :d]


def _fig3(r, seed, n=20000):
    return W.fixed_spectrum(n, np.linspace(1.0, r, D), seed).numpy()


@pytest.mark.parametrize("method", ["svd", "qr"])
@pytest.mark.parametrize("r", [1e-2, 1e-5, 1e-9])
def test_preconditioner(gpu, method, r):
    """The linspace spectra of the preconditioning experiment: the same k
    as the oracle, kappa(A N) within the theorem's xi eta and equal to the
    oracle's, and N N^T (sign-free) equal to the oracle's up to the
    conditioning of the sketch's factor."""
    A = _fig3(r, 21)
    Ag = torch.from_numpy(A).to(gpu)
    N, k = api.lev_precondition(Ag, 9, R_CS, M, 1e-10, method)
    N, k = N.cpu().numpy(), int(k.item())
    No, ko = P.count_gauss_precondition(A, 9, R_CS, M, 1e-10, method)
    assert k == ko == D
    assert np.all(N[:, k:] == 0)
    kg, ko_ = np.linalg.cond(A @ N[:, :k]), np.linalg.cond(A @ No)
    _log(method, r, "kappa(AN)", kg, ko_)
    assert kg <= P.kappa_bound(D, M, 0.2, 0.5) and abs(kg - ko_) <= 1e-6 * ko_
    G, Go = N[:, :k] @ N[:, :k].T, No @ No.T
    err = np.linalg.norm(G - Go) / np.linalg.norm(Go)
    _log("N N^T rel err", err)
    assert err <= 1e-12 / r


def test_preconditioner_rank_deficient_and_wide(gpu):
    """Rank 40 of 60 (both methods find k = 40); the QR method at d = 300
    (the SVD one takes d <= 128)."""
    rng = np.random.default_rng(22)
    B = rng.standard_normal((20000, 40)) @ rng.standard_normal((40, D))
    for method in ("svd", "qr"):
        N, k = api.lev_precondition(torch.from_numpy(B).to(gpu), 3, R_CS, M, 1e-8, method)
        assert int(k.item()) == 40
        assert np.linalg.cond(B @ N.cpu().numpy()[:, :40]) < 20
    A = rng.standard_normal((30000, 300)) * rng.lognormal(0, 2, 300)
    N, k = api.lev_precondition(torch.from_numpy(A).to(gpu), 4, 8192, 600, 1e-10, "qr")
    assert int(k.item()) == 300
    assert np.linalg.cond(A @ N.cpu().numpy()) < 20
    with pytest.raises(api.LevError):
        api.lev_precondition(torch.from_numpy(A).to(gpu), 4, 8192, 600, 1e-10, "svd")


@pytest.mark.parametrize("d", [97, 99, 128])
def test_preconditioner_svd_widths(gpu, d):
    """The Jacobi SVD at odd d (a zero column pads the round-robin
    pairing), past 64 columns (eight elements of a column per lane) and at
    the largest d (W fills 128 KiB of LDS, 64 pairs a round): k,
    kappa(A N) and N N^T against the oracle's SVD."""
    rng = np.random.default_rng(d)
    A = rng.standard_normal((20000, d)) * np.logspace(0, -3, d)
    N, k = api.lev_precondition(_padded(A, torch.float64, gpu), 17, 8192, 2 * d, 1e-10, "svd")
    N, k = N.cpu().numpy(), int(k.item())
    No, ko = P.count_gauss_precondition(A, 17, 8192, 2 * d, 1e-10, "svd")
    assert k == ko == d
    kg, ko_ = np.linalg.cond(A @ N), np.linalg.cond(A @ No)
    _log("svd", d, "kappa(AN)", kg, ko_)
    assert kg < 20 and abs(kg - ko_) <= 1e-6 * ko_
    G, Go = N @ N.T, No @ No.T
    assert np.linalg.norm(G - Go) <= 1e-9 * np.linalg.norm(Go)


@pytest.mark.parametrize("method", ["svd", "qr"])
def test_preconditioner_csr(gpu, method):
    """CSR input (power-law rows, 8 zero columns, so k = 88 of 96): the
    sketch goes through the CSR pass 1; k, kappa(A N) and N N^T against the
    oracle's on the same scipy matrix (FP32 values, exact in FP64)."""
    import scipy.sparse as sp
    n, d, zc = 30000 + 7, 96, 8
    S = W.sparse_power_law(n, d, zc, 41).to_scipy()
    S.sort_indices()
    vals = S.data.astype(np.float32)
    A = api.Csr(torch.from_numpy(S.indptr.astype(np.int64)).to(gpu), torch.from_numpy(S.indices.astype(np.int32)).to(gpu),
                torch.from_numpy(vals).to(gpu), n, d)
    Sh = sp.csr_matrix((vals.astype(np.float64), S.indices, S.indptr), shape=(n, d))
    N, k = api.lev_precondition(A, 13, 8192, 2 * d, 1e-10, method)
    N, k = N.cpu().numpy(), int(k.item())
    No, ko = P.count_gauss_precondition(Sh, 13, 8192, 2 * d, 1e-10, method)
    assert k == ko == d - zc
    assert np.all(N[:, k:] == 0)
    Ad = Sh.toarray()
    kg, ko_ = np.linalg.cond(Ad @ N[:, :k]), np.linalg.cond(Ad @ No)
    _log("csr", method, "kappa(AN)", kg, ko_)
    assert kg < 20 and abs(kg - ko_) <= 1e-6 * ko_
    G, Go = N[:, :k] @ N[:, :k].T, No @ No.T
    assert np.linalg.norm(G - Go) <= 1e-9 * np.linalg.norm(Go)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_lsqr_on_preconditioned_operator(gpu, dtype):
    """LSQR on A N: the GPU's iterates against the oracle's recurrences run
    with the GPU's own N on the same stored A (FP64 arithmetic on both
    sides), and the solution against the least-squares solution."""
    A = _fig3(1e-4, 23).astype(np.float64)
    At = _padded(A, dtype, gpu)
    Ah = At.cpu().to(torch.float64).numpy()
    b = np.random.default_rng(24).standard_normal(A.shape[0])
    N, k = api.lev_precondition(At, 5, R_CS, M, 1e-10, "svd")
    x, hist = api.lev_lsqr(At, N, torch.from_numpy(b).to(gpu), 40)
    x, hist = x.cpu().numpy(), hist.cpu().numpy()
    Nh = N.cpu().numpy()
    xo, ho = P.preconditioned_lsqr(Ah, Nh, b, 40)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _log(dtype, "lsqr vs oracle", rel, "hist", hist[-1], ho[-1])
    assert rel < 1e-9
    np.testing.assert_allclose(hist, ho, rtol=1e-9)
    xs = np.linalg.lstsq(Ah, b, rcond=None)[0]
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,d", [(3001, 37), (4099, 257)])
def test_lsqr_ragged_columns(gpu, dtype, n, d):
    """The passes' column layout at d not a multiple of 4 (the last vector
    of a row half past d) and past one 256-column slice, with a row count
    that leaves the workgroups' row ranges ragged.  Before convergence an
    LSQR iterate moves by ~1e-8 under a rounding-level change of N (the
    oracle alone shows it), so the comparison is at convergence (80 steps
    at kappa(A N) ~ 5): the solution against the oracle's and the
    least-squares one, the residual history against the oracle's."""
    rng = np.random.default_rng(n + d)
    A = rng.standard_normal((n, d)) * rng.uniform(0.2, 5.0, d)
    At = _padded(A, dtype, gpu)
    Ah = At.cpu().to(torch.float64).numpy()
    b = rng.standard_normal(n)
    N, k = api.lev_precondition(At, 9, 4096, 2 * d, 1e-10, "qr")
    assert int(k.item()) == d
    x, hist = api.lev_lsqr(At, N, torch.from_numpy(b).to(gpu), 80)
    x = x.cpu().numpy()
    xo, ho = P.preconditioned_lsqr(Ah, N.cpu().numpy(), b, 80)
    xs = np.linalg.lstsq(Ah, b, rcond=None)[0]
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _log(dtype, n, d, "lsqr ragged vs oracle", rel, "vs lstsq", np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert rel < 1e-9
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    np.testing.assert_allclose(hist.cpu().numpy(), ho, rtol=1e-6)


def test_lsqr_edge_cases(gpu):
    """b = 0 stops at once with x = 0; zero steps give x = 0; the QR
    preconditioner of a rank-deficient A gives a least-squares solution."""
    rng = np.random.default_rng(25)
    A = torch.from_numpy(rng.standard_normal((5000, 16))).to(gpu)
    N, _ = api.lev_precondition(A, 1, 2048, 32, 1e-10, "qr")
    x, h = api.lev_lsqr(A, N, torch.zeros(5000, dtype=torch.float64, device=gpu), 5)
    assert torch.all(x == 0) and torch.all(h == 0)
    x, _ = api.lev_lsqr(A, N, torch.ones(5000, dtype=torch.float64, device=gpu), 0)
    assert torch.all(x == 0)
    B = rng.standard_normal((8000, 10)) @ rng.standard_normal((10, 24))
    Bg = torch.from_numpy(B).to(gpu)
    N, k = api.lev_precondition(Bg, 2, 4096, 48, 1e-8, "qr")
    assert int(k.item()) == 10
    b = rng.standard_normal(8000)
    x, _ = api.lev_lsqr(Bg, N, torch.from_numpy(b).to(gpu), 40)
    xs = np.linalg.lstsq(B, b, rcond=1e-10)[0]
    assert np.linalg.norm(B @ x.cpu().numpy() - b) == pytest.approx(np.linalg.norm(B @ xs - b), rel=1e-10)
