"""The seeded input generators produce the structure their recipes state."""

import numpy as np
import torch

from paper_2105_11004_amd import workloads as W


def test_power_law_alpha_hits_the_mean():
    a = W.power_law_alpha(448, 16.0)
    ell = np.arange(1, 449, dtype=np.float64)
    w = ell ** -a
    assert abs((ell * w).sum() / w.sum() - 16.0) < 1e-9
    assert 1.45 < a < 1.55


def test_sparse_power_law_structure():
    A = W.sparse_power_law(20000, 128, 16, 9)
    rp, ci = A.row_ptr.numpy(), A.col_idx.numpy()
    lens = np.diff(rp)
    assert rp[0] == 0 and rp[-1] == A.nnz == ci.size == A.values.numel()
    assert lens.min() >= 1 and lens.max() <= 112
    assert abs(lens.mean() - 16.0) < 1.0
    zero = set(A.zero_cols.tolist())
    assert len(zero) == 16 and not zero & set(np.unique(ci).tolist())
    for i in range(0, 20000, 997):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    B = W.sparse_power_law(20000, 128, 16, 9)
    assert torch.equal(A.col_idx, B.col_idx) and torch.equal(A.values, B.values)


def test_low_rank_coherent_shape_and_rank():
    A = W.low_rank_coherent(3000, 64, 20, 1).to(torch.float64).numpy()
    s = np.linalg.svd(A, compute_uv=False)
    assert s[19] / s[0] > 1e-6 and s[20] / s[0] < 1e-6
