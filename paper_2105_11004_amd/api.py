"""ctypes binding of liblev (include/lev.h), same names as the C calls.

Argument marshalling only: every step of the estimator runs in the HIP
kernels of liblev.  PyTorch provides device memory (inputs, outputs,
workspace) and the stream (the current stream of the input's device).
There is no fallback: if liblev.so is missing, or a call returns an error,
an exception is raised.
"""

from __future__ import annotations

import ctypes
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p
from dataclasses import dataclass
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "liblev.so"

LEV_OK = 0
STATUS_NAMES = {0: "LEV_OK", -1: "LEV_ERR_ARG", -2: "LEV_ERR_SHAPE", -3: "LEV_ERR_DTYPE",
                -4: "LEV_ERR_FORMAT", -5: "LEV_ERR_WORKSPACE", -6: "LEV_ERR_HIP",
                -7: "LEV_ERR_NOT_SUPPORTED"}
DENSE, CSR = 0, 1
F64, F32, BF16 = 0, 1, 2
AZ = {"native": 0, "fp32": 1, "bf16": 2, "bf16x2": 3, "bf16x3": 4}
WS_SKETCH, WS_ESTIMATE, WS_BACKWARD = 0, 2, 3

# Every symbol the header declares (checked by the CPU tests).
EXPORTED = ["lev_workspace_size", "lev_rank_workspace_size", "lev_state_size", "lev_sketch",
            "lev_rank_estimate", "lev_estimate", "lev_estimate_backward", "lev_debug_hash",
            "lev_debug_buckets", "lev_debug_gaussian", "lev_hash_params", "lev_set_phase_events",
            "lev_status_string", "lev_last_error", "lev_noalloc_max_bytes", "lev_estimate_noalloc",
            "lev_precondition_workspace_size", "lev_precondition", "lev_lsqr_workspace_size", "lev_lsqr",
            "lev_debug_stream_read"]
LEV_STREAM_READ_SINK = 262144
LEV_PHASES = 7
# phase 0 holds no kernels (the Gaussian draws run inside pass 1): its time is
# the cost of two back-to-back events
PHASE_NAMES = ["entry", "pass1_countsketch", "gaussian_transform", "rank_revealing_qr",
               "form_z", "pass2_rownorm"]


class LevMatrix(ctypes.Structure):
    _fields_ = [("format", c_int32), ("dtype", c_int32), ("n", c_int64), ("d", c_int64),
                ("ld", c_int64), ("nnz", c_int64), ("values", c_void_p), ("row_ptr", c_void_p),
                ("col_idx", c_void_p)]


class LevParams(ctypes.Structure):
    _fields_ = [("seed", c_uint64), ("r_cs", c_int64), ("m", c_int64), ("k", c_int64),
                ("zeta", c_double), ("az_precision", c_int32), ("mode", c_int32), ("sketch", c_int32)]


class LevError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: Path | None = None):
    """Loads liblev.so once (torch is imported first so that the HIP runtime
    it ships is the one liblev binds to)."""
    global _lib
    if _lib is not None:
        return _lib
    p = Path(path) if path is not None else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2105_11004_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(str(p))
    vp = c_void_p
    lib.lev_workspace_size.argtypes = [POINTER(LevMatrix), POINTER(LevParams), c_int]
    lib.lev_workspace_size.restype = c_size_t
    lib.lev_rank_workspace_size.argtypes = [c_int64, c_int64]
    lib.lev_rank_workspace_size.restype = c_size_t
    lib.lev_state_size.argtypes = [c_int64, c_int64, c_int64]
    lib.lev_state_size.restype = c_size_t
    lib.lev_sketch.argtypes = [POINTER(LevMatrix), POINTER(LevParams), vp, vp, vp, c_size_t, vp]
    lib.lev_rank_estimate.argtypes = [vp, c_int64, c_int64, c_double, vp, vp, vp, vp, c_size_t, vp]
    lib.lev_estimate.argtypes = [POINTER(LevMatrix), POINTER(LevParams), vp, vp, vp, c_size_t, vp]
    lib.lev_estimate_backward.argtypes = [POINTER(LevMatrix), POINTER(LevParams), vp, vp, vp, vp,
                                          c_size_t, vp]
    lib.lev_debug_hash.argtypes = [c_uint64, c_int64, c_int64, vp, vp, vp]
    lib.lev_debug_buckets.argtypes = [c_uint64, c_int64, c_int64, vp, vp, vp]
    lib.lev_debug_gaussian.argtypes = [c_uint64, c_int, c_int64, c_int64, vp, vp]
    lib.lev_hash_params.argtypes = [c_uint64, c_int64, c_int64, POINTER(c_uint64)]
    lib.lev_noalloc_max_bytes.argtypes = []
    lib.lev_noalloc_max_bytes.restype = c_size_t
    lib.lev_estimate_noalloc.argtypes = [POINTER(LevMatrix), POINTER(LevParams), vp, vp]
    lib.lev_precondition_workspace_size.argtypes = [POINTER(LevMatrix), POINTER(LevParams)]
    lib.lev_precondition_workspace_size.restype = c_size_t
    lib.lev_precondition.argtypes = [POINTER(LevMatrix), POINTER(LevParams), c_int, vp, vp, vp, c_size_t, vp]
    lib.lev_lsqr_workspace_size.argtypes = [POINTER(LevMatrix)]
    lib.lev_lsqr_workspace_size.restype = c_size_t
    lib.lev_lsqr.argtypes = [POINTER(LevMatrix), vp, vp, c_int64, vp, vp, vp, c_size_t, vp]
    lib.lev_debug_stream_read.argtypes = [vp, c_int64, vp, vp]
    lib.lev_set_phase_events.argtypes = [vp, c_int]
    lib.lev_set_phase_events.restype = c_int
    lib.lev_status_string.argtypes = [c_int]
    lib.lev_status_string.restype = ctypes.c_char_p
    lib.lev_last_error.argtypes = []
    lib.lev_last_error.restype = ctypes.c_char_p
    for name in ("lev_sketch", "lev_rank_estimate", "lev_estimate", "lev_estimate_backward",
                 "lev_debug_hash", "lev_debug_buckets", "lev_debug_gaussian", "lev_hash_params",
                 "lev_estimate_noalloc", "lev_debug_stream_read"):
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != LEV_OK:
        raise LevError(status, load_library().lev_last_error().decode())


def _stream(device: torch.device) -> c_void_p:
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> c_void_p:
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(None)


_DTYPES = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


@dataclass
class Csr:
    """A CSR matrix on the device: row_ptr int64[n+1], col_idx int32[nnz]
    (strictly increasing within each row, < d), values[nnz] (float64,
    float32 or bfloat16).  Any object with these five attributes is accepted
    where a Csr is."""
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: torch.Tensor
    n: int
    d: int


def _is_csr(A) -> bool:
    return not isinstance(A, torch.Tensor) and all(hasattr(A, a) for a in ("row_ptr", "col_idx", "values", "n", "d"))


def _as_csr(A):
    if isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr:
        # torch keeps both index arrays in one dtype; the ABI takes int64
        # row pointers and int32 column ids
        return Csr(A.crow_indices().to(torch.int64), A.col_indices().to(torch.int32), A.values(), A.shape[0],
                   A.shape[1])
    return A


def _device(A) -> torch.device:
    A = _as_csr(A)
    return A.values.device if _is_csr(A) else A.device


def _shape(A) -> tuple[int, int]:
    A = _as_csr(A)
    return (int(A.n), int(A.d)) if _is_csr(A) else (A.shape[0], A.shape[1])


def _dtype(A) -> torch.dtype:
    A = _as_csr(A)
    return A.values.dtype if _is_csr(A) else A.dtype


def _matrix(A) -> LevMatrix:
    A = _as_csr(A)
    if _is_csr(A):
        rp, ci, va = A.row_ptr, A.col_idx, A.values
        for name, t in (("row_ptr", rp), ("col_idx", ci), ("values", va)):
            if not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise ValueError(f"CSR {name} must be a contiguous 1-D device tensor")
        if rp.dtype != torch.int64 or ci.dtype != torch.int32:
            raise ValueError("CSR row_ptr must be int64 and col_idx int32")
        if va.dtype not in _DTYPES:
            raise ValueError(f"unsupported dtype {va.dtype}")
        if rp.numel() != int(A.n) + 1 or ci.numel() != va.numel():
            raise ValueError("CSR sizes are inconsistent (row_ptr must have n + 1 entries)")
        return LevMatrix(CSR, _DTYPES[va.dtype], int(A.n), int(A.d), 0, va.numel(), va.data_ptr(), rp.data_ptr(),
                         ci.data_ptr())
    if not A.is_cuda:
        raise ValueError("A must be a device (cuda) tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor with unit column stride")
    if A.dtype not in _DTYPES:
        raise ValueError(f"unsupported dtype {A.dtype}")
    ld = A.stride(0)
    return LevMatrix(DENSE, _DTYPES[A.dtype], A.shape[0], A.shape[1], ld, 0, A.data_ptr(), None, None)


# lev_params.mode: the JL estimate (Algorithm 10), the exact scores of A_K
# (Algorithm 7) or the estimate without the JL step (Pi_2 = I).
MODES = {"jl": 0, "exact": 1, "nojl": 2, "qless": 3}
# lev_params.sketch: the Gaussian stage G (S A) of Algorithm 3, or the SRHT
# F (S A) (the F S composition of Section 4).
SKETCHES = {"gauss": 0, "srht": 1}


def _params(seed, r_cs, m, k, zeta, precision, mode="jl", sketch="gauss") -> LevParams:
    if precision not in AZ:
        raise ValueError(f"precision must be one of {list(AZ)}")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {list(MODES)}")
    if sketch not in SKETCHES:
        raise ValueError(f"sketch must be one of {list(SKETCHES)}")
    return LevParams(int(seed) & ((1 << 64) - 1), int(r_cs), int(m), int(k), float(zeta), AZ[precision],
                     MODES[mode], SKETCHES[sketch])


def _mode(mode: str, exact: bool) -> str:
    return "exact" if exact else mode


def _workspace(nbytes: int, device) -> tuple[torch.Tensor, c_void_p]:
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    aligned = (base + 255) // 256 * 256
    return buf, c_void_p(aligned)


@dataclass
class State:
    """Device blob lev_estimate writes for lev_estimate_backward, plus views
    of its fields (perm, rank, R, Z, A~)."""
    blob: torch.Tensor
    d: int
    m: int
    k: int

    def _f64(self, offset: int, count: int) -> torch.Tensor:
        return self.blob[offset:offset + 8 * count].view(torch.float64)

    @staticmethod
    def layout(d: int, m: int, k: int):
        al = lambda x: (x + 255) // 256 * 256  # noqa: E731
        off = {}
        pos = 0
        for name, nbytes in (("header", 64), ("perm", 4 * d), ("R", 8 * d * d), ("Z", 8 * d * k),
                             ("At", 8 * m * d)):
            off[name] = pos
            pos += al(nbytes)
        return off

    @property
    def rank(self) -> torch.Tensor:
        off = self.layout(self.d, self.m, self.k)["header"]
        return self.blob[off + 32:off + 40].view(torch.int64)

    @property
    def error(self) -> torch.Tensor:
        """The device error word (0: every bounded wait ended normally)."""
        off = self.layout(self.d, self.m, self.k)["header"]
        return self.blob[off + 40:off + 44].view(torch.int32)

    @property
    def perm(self) -> torch.Tensor:
        off = self.layout(self.d, self.m, self.k)["perm"]
        return self.blob[off:off + 4 * self.d].view(torch.int32)

    @property
    def R(self) -> torch.Tensor:
        off = self.layout(self.d, self.m, self.k)["R"]
        return self._f64(off, self.d * self.d).view(self.d, self.d)

    @property
    def Z(self) -> torch.Tensor:
        off = self.layout(self.d, self.m, self.k)["Z"]
        return self._f64(off, self.d * self.k).view(self.d, self.k)

    @property
    def At(self) -> torch.Tensor:
        off = self.layout(self.d, self.m, self.k)["At"]
        return self._f64(off, self.m * self.d).view(self.m, self.d)


def _aligned_blob(nbytes: int, device) -> torch.Tensor:
    """A uint8 tensor of nbytes whose data pointer is 256-byte aligned."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes)]


def lev_workspace_size(A, seed, r_cs, m, k, zeta, precision="native", which=WS_ESTIMATE) -> int:
    lib = load_library()
    A = _as_csr(A)
    mat, par = _matrix(A), _params(seed, r_cs, m, k, zeta, precision)
    return int(lib.lev_workspace_size(ctypes.byref(mat), ctypes.byref(par), which))


def lev_sketch(A, seed: int, r_cs: int, m: int, return_sa: bool = False, sketch: str = "gauss"):
    """Algorithm 3: A~ = G (S A) (m x d, FP64), or F (S A) with the SRHT F
    (sketch="srht"); optionally also S A.  A is a dense device tensor or a
    CSR matrix (Csr, or a torch sparse_csr tensor with int64 row pointers
    and int32 column indices)."""
    lib = load_library()
    A = _as_csr(A)  # held until the call returns: it owns converted index arrays
    dev, (_, d) = _device(A), _shape(A)
    prec = "fp32" if (_dtype(A) == torch.bfloat16 and not _is_csr(_as_csr(A))) else "native"
    mat, par = _matrix(A), _params(seed, r_cs, m, 1, 0.0, prec, sketch=sketch)
    nbytes = lib.lev_workspace_size(ctypes.byref(mat), ctypes.byref(par), WS_SKETCH)
    if nbytes == 0:
        _check(lib.lev_sketch(ctypes.byref(mat), ctypes.byref(par), None, None, None, 0, None))
    _, ws = _workspace(nbytes, dev)
    At = torch.empty(m, d, dtype=torch.float64, device=dev)
    SA = torch.empty(r_cs, d, dtype=torch.float64, device=dev) if return_sa else None
    _check(lib.lev_sketch(ctypes.byref(mat), ctypes.byref(par), _ptr(At), _ptr(SA), ws, nbytes, _stream(dev)))
    return (At, SA) if return_sa else At


def lev_rank_estimate(At: torch.Tensor, zeta: float):
    """Algorithm 4 steps 2-3 on an m x d FP64 sketch: (perm int32[d],
    R d x d, rank int64[1]), all on the device."""
    lib = load_library()
    if At.dtype != torch.float64 or At.dim() != 2 or not At.is_contiguous() or not At.is_cuda:
        raise ValueError("At must be a contiguous m x d float64 device tensor")
    m, d = At.shape
    nbytes = lib.lev_rank_workspace_size(m, d)
    if nbytes == 0:
        raise LevError(-2, f"invalid sketch shape {m} x {d}")
    _, ws = _workspace(nbytes, At.device)
    perm = torch.empty(d, dtype=torch.int32, device=At.device)
    R = torch.empty(d, d, dtype=torch.float64, device=At.device)
    rank = torch.empty(1, dtype=torch.int64, device=At.device)
    _check(lib.lev_rank_estimate(_ptr(At), m, d, float(zeta), _ptr(perm), _ptr(R), _ptr(rank), ws, nbytes,
                                 _stream(At.device)))
    return perm, R, rank


def lev_estimate(A, seed: int, r_cs: int, m: int, k: int, zeta: float,
                 precision: str = "native", return_state: bool = False, exact: bool = False,
                 mode: str = "jl", sketch: str = "gauss"):
    """Algorithm 10 (LS-HRN-approx): theta~ (FP64 for FP64 A, else FP32).
    A is a dense device tensor or a CSR matrix (see lev_sketch).
    mode="exact" (or exact=True) runs Algorithm 7 (LS-HRN-exact) instead:
    the exact leverage scores of the columns K the sketch selects;
    mode="nojl" the estimate without the JL step, ||e_i^T A_K R11^{-1}||^2
    (both ignore k); mode="qless" Algorithm 6, the exact scores from a Q-less
    pivoted QR of A itself with k as its step cap (no sketch).  Only the JL
    estimate has a state.  sketch="srht" takes the SRHT F (S A)
    in place of the Gaussian stage G (S A)."""
    lib = load_library()
    A = _as_csr(A)  # held until the call returns: it owns converted index arrays
    dev, (n, d), dt = _device(A), _shape(A), _dtype(A)
    mat, par = _matrix(A), _params(seed, r_cs, m, k, zeta, precision, _mode(mode, exact), sketch)
    nbytes = lib.lev_workspace_size(ctypes.byref(mat), ctypes.byref(par), WS_ESTIMATE)
    if nbytes == 0:
        _check(lib.lev_estimate(ctypes.byref(mat), ctypes.byref(par), None, None, None, 0, None))
    _, ws = _workspace(nbytes, dev)
    out_dtype = torch.float64 if dt == torch.float64 else torch.float32
    theta = torch.empty(n, dtype=out_dtype, device=dev)
    state = None
    if return_state:
        state = State(_aligned_blob(lib.lev_state_size(d, m, k), dev), d, m, k)
    _check(lib.lev_estimate(ctypes.byref(mat), ctypes.byref(par), _ptr(theta),
                            _ptr(state.blob) if state is not None else None, ws, nbytes, _stream(dev)))
    return (theta, state) if return_state else theta


def lev_estimate_noalloc(A, seed: int, r_cs: int, m: int, k: int, zeta: float, precision: str = "native",
                         theta: torch.Tensor | None = None):
    """lev_estimate through the entry point that allocates no device memory
    (its workspace is the library's static scratch array).  theta may be a
    preallocated output; it is allocated here only when it is None."""
    lib = load_library()
    A = _as_csr(A)
    dev, (n, _), dt = _device(A), _shape(A), _dtype(A)
    mat, par = _matrix(A), _params(seed, r_cs, m, k, zeta, precision)
    if theta is None:
        theta = torch.empty(n, dtype=torch.float64 if dt == torch.float64 else torch.float32, device=dev)
    _check(lib.lev_estimate_noalloc(ctypes.byref(mat), ctypes.byref(par), _ptr(theta), _stream(dev)))
    return theta


PRECOND = {"qr": 0, "svd": 1}


def lev_precondition(A, seed: int, r_cs: int, m: int, zeta: float, method: str = "svd", sketch: str = "gauss"):
    """Algorithm 11: (N, k) with N the d x d FP64 right preconditioner
    (columns past k zero) from the sketch of A; method "svd" (N = V_k
    Sigma_k^{-1}, d <= 128) or "qr" (N = P R11^{-1}).  k stays a device
    tensor (-1 if a bounded wait ran out)."""
    if method not in PRECOND:
        raise ValueError(f"method must be one of {list(PRECOND)}")
    lib = load_library()
    A = _as_csr(A)
    dev, (_, d) = _device(A), _shape(A)
    mat, par = _matrix(A), _params(seed, r_cs, m, 1, zeta, "native", sketch=sketch)
    nbytes = lib.lev_precondition_workspace_size(ctypes.byref(mat), ctypes.byref(par))
    if nbytes == 0:
        _check(lib.lev_precondition(ctypes.byref(mat), ctypes.byref(par), PRECOND[method], None, None, None, 0,
                                    None))
    _, ws = _workspace(nbytes, dev)
    N = torch.empty(d, d, dtype=torch.float64, device=dev)
    k = torch.empty(1, dtype=torch.int64, device=dev)
    _check(lib.lev_precondition(ctypes.byref(mat), ctypes.byref(par), PRECOND[method], _ptr(N), _ptr(k), ws,
                                nbytes, _stream(dev)))
    return N, k


def lev_lsqr(A: torch.Tensor, N: torch.Tensor, b: torch.Tensor, iters: int):
    """LSQR on A N from y = 0 for `iters` steps; returns x = N y (FP64, d)
    and the residual-norm estimate after each step (FP64, iters)."""
    lib = load_library()
    dev, (n, d) = _device(A), _shape(A)
    mat = _matrix(A)
    nbytes = lib.lev_lsqr_workspace_size(ctypes.byref(mat))
    if nbytes == 0:
        _check(lib.lev_lsqr(ctypes.byref(mat), None, None, 0, None, None, None, 0, None))
    _, ws = _workspace(nbytes, dev)
    N = N.to(torch.float64).contiguous()
    b = b.to(torch.float64).contiguous()
    x = torch.empty(d, dtype=torch.float64, device=dev)
    hist = torch.empty(max(int(iters), 1), dtype=torch.float64, device=dev)
    _check(lib.lev_lsqr(ctypes.byref(mat), _ptr(N), _ptr(b), int(iters), _ptr(x), _ptr(hist), ws, nbytes,
                        _stream(dev)))
    return x, hist[:int(iters)]


class EstimatePlan:
    """Pre-allocated workspace and outputs for repeated lev_estimate calls on
    same-shaped inputs (what the benchmark times)."""

    def __init__(self, A, seed, r_cs, m, k, zeta, precision="native", exact=False, mode="jl", sketch="gauss"):
        self.lib = load_library()
        A = _as_csr(A)  # kept in self.A: the pointers below refer to its arrays
        self.mat, self.par = _matrix(A), _params(seed, r_cs, m, k, zeta, precision, _mode(mode, exact), sketch)
        self.nbytes = self.lib.lev_workspace_size(ctypes.byref(self.mat), ctypes.byref(self.par), WS_ESTIMATE)
        if self.nbytes == 0:
            _check(self.lib.lev_estimate(ctypes.byref(self.mat), ctypes.byref(self.par), None, None, None, 0,
                                         None))
        self.device = _device(A)
        self._buf, self.ws = _workspace(self.nbytes, self.device)
        out_dtype = torch.float64 if _dtype(A) == torch.float64 else torch.float32
        self.theta = torch.empty(_shape(A)[0], dtype=out_dtype, device=self.device)
        self.A = A

    def run(self, stream=None):
        s = c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        _check(self.lib.lev_estimate(ctypes.byref(self.mat), ctypes.byref(self.par), _ptr(self.theta), None,
                                     self.ws, self.nbytes, s))
        return self.theta


class BackwardPlan:
    """Pre-allocated workspace, state and gradient for repeated
    lev_estimate_backward calls after an EstimatePlan's forward (the
    benchmark's backward step)."""

    def __init__(self, plan: "EstimatePlan", w: torch.Tensor):
        self.plan, self.lib = plan, plan.lib
        A = plan.A
        n, d = _shape(A)
        p = plan.par
        self.state = State(_aligned_blob(self.lib.lev_state_size(d, p.m, p.k), plan.device), d, p.m, p.k)
        self.nbytes = self.lib.lev_workspace_size(ctypes.byref(plan.mat), ctypes.byref(p), WS_BACKWARD)
        if self.nbytes == 0:
            _check(self.lib.lev_estimate_backward(ctypes.byref(plan.mat), ctypes.byref(p), None, None, None, None,
                                                  0, None))
        self._buf, self.ws = _workspace(self.nbytes, plan.device)
        self.w = w.contiguous()
        self.grad = torch.empty(n, A.stride(0), dtype=A.dtype, device=plan.device)
        # the forward that fills the state
        _check(self.lib.lev_estimate(ctypes.byref(plan.mat), ctypes.byref(p), _ptr(plan.theta), _ptr(self.state.blob),
                                     plan.ws, plan.nbytes, _stream(plan.device)))

    def run(self):
        p = self.plan
        _check(self.lib.lev_estimate_backward(ctypes.byref(p.mat), ctypes.byref(p.par), _ptr(self.state.blob),
                                              _ptr(self.w), _ptr(self.grad), self.ws, self.nbytes,
                                              _stream(p.device)))
        return self.grad


def lev_set_phase_events(events):
    """Registers LEV_PHASES torch.cuda.Event objects (already recorded once,
    so that they exist) for the phase boundaries of following lev_estimate
    calls on this thread; None stops recording."""
    lib = load_library()
    if events is None:
        _check(lib.lev_set_phase_events(None, 0))
        return
    if len(events) != LEV_PHASES:
        raise ValueError(f"need {LEV_PHASES} events")
    arr = (c_void_p * LEV_PHASES)(*[c_void_p(e.cuda_event) for e in events])
    _check(lib.lev_set_phase_events(arr, LEV_PHASES))


def lev_debug_hash(seed: int, n: int, r_cs: int, device="cuda"):
    lib = load_library()
    h = torch.empty(n, dtype=torch.int64, device=device)
    s = torch.empty(n, dtype=torch.int8, device=device)
    _check(lib.lev_debug_hash(int(seed) & ((1 << 64) - 1), n, r_cs, _ptr(h), _ptr(s),
                              _stream(torch.device(device))))
    return h, s


def lev_debug_buckets(seed: int, n: int, r_cs: int, device="cuda"):
    lib = load_library()
    off = torch.empty(r_cs + 1, dtype=torch.int64, device=device)
    rows = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    _check(lib.lev_debug_buckets(int(seed) & ((1 << 64) - 1), n, r_cs, _ptr(off), _ptr(rows),
                                 _stream(torch.device(device))))
    return off, rows[:n]


def lev_hash_params(seed: int, n: int, r_cs: int) -> dict:
    """The hash and sign coefficients liblev derives from a seed (host
    only, no GPU needed): P, a, c, c0..c3."""
    lib = load_library()
    out = (c_uint64 * 7)()
    _check(lib.lev_hash_params(int(seed) & ((1 << 64) - 1), int(n), int(r_cs), out))
    return dict(zip(("P", "a", "c", "c0", "c1", "c2", "c3"), [int(v) for v in out]))


def lev_debug_gaussian(seed: int, which: int, rows: int, cols: int, device="cuda"):
    lib = load_library()
    out = torch.empty(rows, cols, dtype=torch.float64, device=device)
    _check(lib.lev_debug_gaussian(int(seed) & ((1 << 64) - 1), which, rows, cols, _ptr(out),
                                  _stream(torch.device(device))))
    return out


def lev_debug_stream_read(buf: torch.Tensor, nbytes: int = None, sink: torch.Tensor = None,
                          stream=None) -> torch.Tensor:
    """One streaming read of the first nbytes (default: all, rounded down to
    16) of a device tensor's storage; returns the per-thread checksums
    (int32, LEV_STREAM_READ_SINK).  stream: a torch stream (default: the
    current one)."""
    lib = load_library()
    if nbytes is None:
        nbytes = buf.numel() * buf.element_size() // 16 * 16
    if sink is None:
        sink = torch.empty(LEV_STREAM_READ_SINK, dtype=torch.int32, device=buf.device)
    st = (stream or torch.cuda.current_stream(buf.device)).cuda_stream
    _check(lib.lev_debug_stream_read(_ptr(buf), int(nbytes), _ptr(sink), ctypes.c_void_p(st)))
    return sink


def lev_estimate_backward(A, state: State, w: torch.Tensor, seed: int, r_cs: int, m: int, k: int, zeta: float,
                          precision: str = "native") -> torch.Tensor:
    """d(w^T theta~)/dA at the sketch, pivots and rank recorded in `state`
    (the blob lev_estimate returned for the same A and parameters).  Dense
    FP32/FP64 A; w has A's dtype and n entries; the gradient has A's dtype
    and shape."""
    lib = load_library()
    A = _as_csr(A)
    mat, par = _matrix(A), _params(seed, r_cs, m, k, zeta, precision)
    nbytes = lib.lev_workspace_size(ctypes.byref(mat), ctypes.byref(par), WS_BACKWARD)
    if nbytes == 0:
        _check(lib.lev_estimate_backward(ctypes.byref(mat), ctypes.byref(par), None, None, None, None, 0, None))
    n, d = _shape(A)
    dev = _device(A)
    if not isinstance(w, torch.Tensor) or w.device != dev or w.dtype != _dtype(A) or w.numel() != n:
        raise ValueError("w must be a device tensor of A's dtype with n entries")
    w = w.contiguous()
    _, ws = _workspace(nbytes, dev)
    ld = A.stride(0)
    g = torch.empty(n, ld, dtype=A.dtype, device=dev)
    _check(lib.lev_estimate_backward(ctypes.byref(mat), ctypes.byref(par), _ptr(state.blob), _ptr(w), _ptr(g), ws,
                                     nbytes, _stream(dev)))
    return g[:, :d]


class LevEstimate(torch.autograd.Function):
    """theta~ = LS-HRN-approx(A) as a differentiable op: the forward keeps the
    state blob (pivots, rank, R, Z, A~), the backward calls the adjoint
    kernels with w = the incoming gradient (sketch, pivots and rank fixed)."""

    @staticmethod
    def forward(ctx, A, seed, r_cs, m, k, zeta, precision="native"):
        theta, state = lev_estimate(A, seed, r_cs, m, k, zeta, precision=precision, return_state=True)
        ctx.save_for_backward(A)
        ctx.state = state
        ctx.params = (seed, r_cs, m, k, zeta, precision)
        return theta

    @staticmethod
    def backward(ctx, grad_theta):
        (A,) = ctx.saved_tensors
        w = grad_theta.to(A.dtype).contiguous()
        gA = lev_estimate_backward(A, ctx.state, w, *ctx.params)
        return gA, None, None, None, None, None, None


def estimate(A: torch.Tensor, seed: int, r_cs: int, m: int, k: int, zeta: float, precision: str = "native"):
    """theta~ with autograd support (see LevEstimate)."""
    return LevEstimate.apply(A, seed, r_cs, m, k, zeta, precision)
