"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws input matrices only; it holds none of the estimator's
arithmetic and is shared by the tests (GPU path and CPU oracle alike) and
the benchmark.  Generation runs on the device given (CPU for small cases,
the GPU for the large ones, where CPU generation would dominate the run);
the same (recipe, seed, device type) gives the same matrix.

Recipes (sizes as in the workload table of the design notes):
  * dense_gaussian   -- A_ij ~ N(0,1) (full rank).
  * low_rank_coherent -- A = U V with U n x rank, V rank x d i.i.d. N(0,1),
    then a seeded 1% of the rows scaled by 1e3 (high coherence).
  * row_scaled_bf16  -- A_ij = N(0,1) * l_i, l_i ~ lognormal(0,1), stored
    in BF16 (round to nearest even).
  * fixed_spectrum   -- A = U diag(sigma) V^T with Haar-like U, V and a
    prescribed singular value list (the fixed_svd matrices of Section 7).
  * sparse_power_law -- CSR rows with power-law lengths on [1, live] (mean
    16 nonzeros), the columns of each row uniform without replacement over
    the live columns (all but a seeded set of zero columns), values N(0,1).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def dense_gaussian(n: int, d: int, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    return torch.randn(n, d, generator=g, dtype=torch.float32 if dtype == torch.bfloat16 else dtype,
                       device=device).to(dtype)


def low_rank_coherent(n: int, d: int, rank: int, seed: int, heavy_frac: float = 0.01,
                      heavy_scale: float = 1e3, dtype=torch.float32, device="cpu",
                      chunk: int = 1 << 18) -> torch.Tensor:
    g = _gen(seed, device)
    V = torch.randn(rank, d, generator=g, dtype=torch.float64, device=device)
    A = torch.empty(n, d, dtype=dtype, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        U = torch.randn(hi - lo, rank, generator=g, dtype=torch.float64, device=device)
        A[lo:hi] = (U @ V).to(dtype)
    n_heavy = int(round(heavy_frac * n))
    if n_heavy > 0:
        rows = torch.randperm(n, generator=g, device=device)[:n_heavy]
        A[rows] = (A[rows].to(torch.float64) * heavy_scale).to(dtype)
    return A


def row_scaled_bf16(n: int, d: int, seed: int, device="cpu", chunk: int = 1 << 18) -> torch.Tensor:
    g = _gen(seed, device)
    A = torch.empty(n, d, dtype=torch.bfloat16, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        scale = torch.exp(torch.randn(hi - lo, 1, generator=g, dtype=torch.float32, device=device))
        A[lo:hi] = (torch.randn(hi - lo, d, generator=g, dtype=torch.float32, device=device) * scale).to(torch.bfloat16)
    return A


def fixed_spectrum(n: int, sigma, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """U diag(sigma) V^T with U, V from QR of Gaussians (Section 7 recipe)."""
    g = _gen(seed, device)
    sigma = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    d = sigma.numel()
    U, _ = torch.linalg.qr(torch.randn(n, d, generator=g, dtype=torch.float64, device=device))
    V, _ = torch.linalg.qr(torch.randn(d, d, generator=g, dtype=torch.float64, device=device))
    return ((U * sigma) @ V.T).to(dtype)


def power_law_alpha(live: int, mean: float) -> float:
    """Exponent alpha of P(l) ~ l^-alpha on [1, live] whose mean is `mean`
    (bisection; the mean decreases monotonically in alpha)."""
    ell = np.arange(1, live + 1, dtype=np.float64)
    lo, hi = 0.0, 8.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        w = ell ** (-mid)
        if (ell * w).sum() / w.sum() > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclass
class CsrHost:
    """CSR matrix as torch tensors (row_ptr int64[n+1], col_idx int32[nnz],
    values[nnz]) on one device."""
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: torch.Tensor
    n: int
    d: int
    zero_cols: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def to(self, device) -> "CsrHost":
        return CsrHost(self.row_ptr.to(device), self.col_idx.to(device), self.values.to(device), self.n, self.d,
                       self.zero_cols.to(device))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values.cpu().to(torch.float64).numpy(), self.col_idx.cpu().numpy(),
                              self.row_ptr.cpu().numpy()), shape=(self.n, self.d))


def sparse_power_law(n: int, d: int, n_zero_cols: int, seed: int, mean_nnz: float = 16.0,
                     dtype=torch.float32, device="cpu", chunk: int = 1 << 15) -> CsrHost:
    """CSR with a seeded set of n_zero_cols all-zero columns; row lengths l in
    [1, live] (live = d - n_zero_cols) with P(l) ~ l^-alpha, alpha set so the
    mean is mean_nnz; each row's columns are l distinct live columns drawn
    uniformly (the l smallest of live random keys), sorted; values N(0,1)."""
    g = _gen(seed, device)
    perm = torch.randperm(d, generator=g, device=device)
    zero_cols = torch.sort(perm[:n_zero_cols]).values
    is_live = torch.ones(d, dtype=torch.bool, device=device)
    is_live[zero_cols] = False
    live = torch.nonzero(is_live).flatten().to(torch.int32)
    n_live = int(live.numel())
    alpha = power_law_alpha(n_live, mean_nnz)
    w = torch.arange(1, n_live + 1, dtype=torch.float64, device=device) ** (-alpha)
    cdf = torch.cumsum(w / w.sum(), 0)
    cdf[-1] = 1.0
    u = torch.rand(n, generator=g, dtype=torch.float64, device=device)
    lengths = torch.searchsorted(cdf, u, right=True).clamp_(max=n_live - 1) + 1
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(lengths, 0, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_idx = torch.empty(nnz, dtype=torch.int32, device=device)
    ar = torch.arange(n_live, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        keys = torch.rand(hi - lo, n_live, generator=g, dtype=torch.float64, device=device)
        order = torch.argsort(keys, dim=1)
        sel = ar[None, :] < lengths[lo:hi, None]
        mask = torch.zeros_like(sel)
        mask.scatter_(1, order, sel)  # exactly l_i columns per row
        cols = torch.nonzero(mask)[:, 1]  # row-major: ascending within a row
        col_idx[int(row_ptr[lo]):int(row_ptr[hi])] = live[cols]
    values = torch.randn(nnz, generator=g, dtype=torch.float32, device=device).to(dtype)
    return CsrHost(row_ptr, col_idx, values, n, d, zero_cols)


# Workload table: the shapes of the paper's sketches at the sizes the tests
# and the benchmark run.
CONFIGS = {
    "dense_f64_4096x64": dict(n=4096, d=64, dtype="f64", r_cs=1024, m=256, k=32, zeta=1e-10),
    "dense_f32_1Mx256_rank128": dict(n=1 << 20, d=256, rank=128, dtype="f32", r_cs=4096, m=512, k=48, zeta=1e-5),
    "csr_f32_8Mx512": dict(n=1 << 23, d=512, zero_cols=64, dtype="f32", r_cs=8192, m=1024, k=64, zeta=1e-5),
    "dense_bf16_4Mx1024": dict(n=1 << 22, d=1024, dtype="bf16", r_cs=16384, m=2048, k=64, zeta=1e-3),
    "dense_f32_1Mx256_rank192_bwd": dict(n=1 << 20, d=256, rank=192, dtype="f32", r_cs=4096, m=512, k=48, zeta=1e-5),
    # LS-HRN-exact (Algorithm 7) at scale: an FP32 Gaussian; k is unused there
    "dense_f32_1Mx64_exact": dict(n=1 << 20, d=64, dtype="f32", r_cs=4096, m=128, k=32, zeta=1e-5),
    # Algorithm 6's regime (rank well below sqrt(d)): the recipe of the
    # 2^20 x 256 workload at rank 16; k is the Q-less QR's step cap there
    "dense_f32_1Mx256_rank16": dict(n=1 << 20, d=256, rank=16, dtype="f32", r_cs=4096, m=512, k=32, zeta=1e-5),
}

# A case at the sizes the theorems ask for (the end-to-end (1 +- eps) check):
# n = 4096, d = 8, a CountSketch of at least the OSE size for eps = 0.5,
# delta = 1/3 ((d^2 + d) / (delta (2 eps - eps^2)^2) = 384 rows, Section 3),
# a Gaussian stage of m = 64 r >= 30 r rows (distortion about sqrt(r / m),
# the subspace embedding the bound of Section 5 composes with) and the JL
# bound for eps = 0.5 (4 ln n / (eps^2 / 2 - eps^3 / 3) = 400 columns).
THEORY_SIZED = dict(n=4096, d=8, r_cs=512, m=512, k=400, eps=0.5, delta=1 / 3)


def theory_sized_matrix() -> np.ndarray:
    """FP64 4096 x 8 Gaussian with lognormal(0, 1) row scales."""
    rng = np.random.default_rng(21)
    n, d = THEORY_SIZED["n"], THEORY_SIZED["d"]
    return rng.standard_normal((n, d)) * rng.lognormal(0, 1, (n, 1))


def sketch_seed(cfg_index: int) -> int:
    return 2000 + cfg_index


def data_seed(cfg_index: int) -> int:
    return 1000 + cfg_index


def expected_bias(m: int, r: int, r_cs: int) -> float:
    """Predicted mean of theta~/theta at a given sketch size (inverse-Wishart
    mean of the Gaussian stage times the CountSketch collision factor); a
    reporting aid, not part of the estimator."""
    if m - r - 1 <= 0 or r_cs <= r:
        return math.inf
    return m / (m - r - 1) * r_cs / (r_cs - r)
