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
  * sparse_power_law -- CSR rows with power-law lengths on [1, live], the
    columns of each row uniform without replacement over the live columns
    (all but a seeded set of zero columns), values N(0,1).
"""

from __future__ import annotations

import math

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


def power_law_lengths(n: int, live: int, alpha: float, seed: int) -> np.ndarray:
    """Row lengths l in [1, live] with P(l) proportional to l^-alpha."""
    rng = np.random.default_rng(seed)
    ell = np.arange(1, live + 1, dtype=np.float64)
    p = ell ** (-alpha)
    p /= p.sum()
    return rng.choice(np.arange(1, live + 1), size=n, p=p).astype(np.int64)


def sparse_power_law(n: int, d: int, n_zero_cols: int, alpha: float, seed: int,
                     dtype=np.float32):
    """CSR (row_ptr int64, col_idx int32 sorted per row, values) on the host.

    Each row draws its length from the truncated power law, then that many
    distinct columns uniformly from the live columns (random keys, take the
    smallest), sorted ascending.
    """
    rng = np.random.default_rng(seed + 1)
    zero_cols = np.sort(rng.choice(d, size=n_zero_cols, replace=False))
    live = np.setdiff1d(np.arange(d), zero_cols).astype(np.int32)
    lengths = power_law_lengths(n, live.size, alpha, seed)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_idx = np.empty(nnz, dtype=np.int32)
    # group rows by length so each group is one vectorised draw
    for ell in np.unique(lengths):
        rows = np.nonzero(lengths == ell)[0]
        for lo in range(0, rows.size, 1 << 16):
            rr = rows[lo:lo + (1 << 16)]
            keys = rng.random((rr.size, live.size), dtype=np.float32)
            pick = np.argpartition(keys, ell - 1, axis=1)[:, :ell] if ell < live.size else \
                np.tile(np.arange(live.size), (rr.size, 1))
            cols = np.sort(live[pick], axis=1)
            starts = row_ptr[rr]
            idx = starts[:, None] + np.arange(ell)[None, :]
            col_idx[idx.ravel()] = cols.ravel()
    values = rng.standard_normal(nnz, dtype=np.float64).astype(dtype)
    return row_ptr, col_idx, values, zero_cols


# Workload table: the shapes of the paper's sketches at the sizes the tests
# and the benchmark run.
CONFIGS = {
    "dense_f64_4096x64": dict(n=4096, d=64, dtype="f64", r_cs=1024, m=256, k=32, zeta=1e-10),
    "dense_f32_1Mx256_rank128": dict(n=1 << 20, d=256, rank=128, dtype="f32", r_cs=4096, m=512, k=48, zeta=1e-5),
    "csr_f32_8Mx512": dict(n=1 << 23, d=512, dtype="f32", r_cs=8192, m=1024, k=64, zeta=1e-5),
    "dense_bf16_4Mx1024": dict(n=1 << 22, d=1024, dtype="bf16", r_cs=16384, m=2048, k=64, zeta=1e-3),
    "dense_f32_1Mx256_rank192_bwd": dict(n=1 << 20, d=256, rank=192, dtype="f32", r_cs=4096, m=512, k=48, zeta=1e-5),
}


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
