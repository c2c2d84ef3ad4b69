"""The entry point that allocates nothing (lev_estimate_noalloc) against
lev_estimate on the same inputs: three calls in a row on one GPU, each
smaller than the one before, so every call after the first runs on scratch
memory that still holds the previous call's contents.  The two entry points
run the same kernels in the same order, so their results are compared bit
for bit (stricter than the 1e-4 / 1e-9 bars of the parity tests)."""

import sys

import pytest
import torch

from paper_2105_11004_amd import api
from paper_2105_11004_amd import workloads as W


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    # (name, A builder, r_cs, m, k, zeta, seed): d > 256 (panel pivoting and
    # its zero-filled progress flags), the FP32 benchmark shape at a smaller
    # n, then the small FP64 case
    ("fp64 3000x300", lambda: W.dense_gaussian(3000, 300, 31, dtype=torch.float64), 2048, 384, 40, 1e-10, 41),
    ("fp32 65549x256 rank 128", lambda: W.low_rank_coherent(65536 + 13, 256, 128, 1002), 4096, 512, 48, 1e-5, 2002),
    ("fp64 4096x64", lambda: W.dense_gaussian(4096, 64, 1001, dtype=torch.float64), 1024, 256, 32, 1e-10, 2001),
]


@pytest.mark.gpu
def test_noalloc_matches_lev_estimate_on_consecutive_calls(gpu):
    lib = api.load_library()
    assert lib.lev_noalloc_max_bytes() == 64 << 20
    for name, make, r_cs, m, k, zeta, seed in CASES:
        _log("noalloc case", name)
        A = make().to(gpu)
        ref, st = api.lev_estimate(A, seed, r_cs, m, k, zeta, return_state=True)
        got = api.lev_estimate_noalloc(A, seed, r_cs, m, k, zeta)
        torch.cuda.synchronize()
        assert int(st.error.item()) == 0
        assert got.dtype == ref.dtype and got.shape == ref.shape
        assert torch.equal(got, ref), (name, (got - ref).abs().max().item())
        # and once more on the same scratch: same bits
        again = api.lev_estimate_noalloc(A, seed, r_cs, m, k, zeta)
        torch.cuda.synchronize()
        assert torch.equal(again, ref), name


def test_noalloc_refuses_problems_beyond_its_scratch():
    """Checked on the host before the device is touched (runs without a GPU)."""
    import ctypes
    lib = api.load_library()
    c = W.CONFIGS["dense_bf16_4Mx1024"]
    mat = api.LevMatrix(api.DENSE, api.BF16, c["n"], c["d"], c["d"], 0, 4096, None, None)
    par = api.LevParams(1, c["r_cs"], c["m"], c["k"], c["zeta"], 0, 0, 0)
    assert lib.lev_workspace_size(ctypes.byref(mat), ctypes.byref(par), api.WS_ESTIMATE) > lib.lev_noalloc_max_bytes()
    st = lib.lev_estimate_noalloc(ctypes.byref(mat), ctypes.byref(par), ctypes.c_void_p(4096), None)
    assert st == -5  # LEV_ERR_WORKSPACE
    assert b"static scratch" in lib.lev_last_error()
