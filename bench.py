"""Benchmark of the rSLS estimator (LS-HRN-approx) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision auto|native|fp32|bf16|bf16x2|bf16x3]
                    [--no-accuracy] [--no-cpu-baseline] [--mode jl|exact|nojl]
                    [--sketch gauss|srht] [--precondition]

One step = one lev_estimate call over the whole workload resident in HBM:
the Gaussian draws and pass 1 (CountSketch S A), the Gaussian transform, the
rank-revealing factorisation, Z = R11^{-1} G_k and pass 2 (theta~); for the
backward workload (name ending in _bwd) also the adjoint of w^T theta~.
--mode exact times Algorithm 7 instead (the exact scores of A_K from B =
A_K^T A_K), --mode nojl the estimate without the JL step (Pi_2 = I);
--sketch srht replaces the Gaussian stage G (S A) by the SRHT F (S A).
--precondition runs Section 6's experiment instead (kappa(A N) of
Algorithm 11's preconditioner over the linspace spectra, and LSQR timing).
Prints one JSON line with rows/s, the per-phase times and rooflines (the
headline `roofline` is the dominant kernel's -- the longer pass over A --
measured live with the HIP events liblev records on its own stream; the
slowest phase overall is reported beside it as `slowest_phase`), the accuracy of theta~ on sampled
rows (against the oracle's FP64 estimator with the same sketch, and against
the exact scores; for BF16 storage every BF16 form side by side), and the
CPU oracle timed on a bounded sample of the same workload.

HBM traffic of the passes (rocprofv3 counters, one process per counter):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o fetch -- python3 bench.py --traffic-run [--workload NAME]
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o write -- python3 bench.py --traffic-run [--workload NAME]
    python3 bench.py --traffic-summarize OUT/fetch OUT/write [--workload NAME]

A traffic run first copies a 1 GiB device buffer (a plain copy kernel that
reads and writes exactly 1 GiB: the calibration of each counter), then runs
lev_estimate twice; the summary scales each pass's counter by the copy's
factor and stores bytes per launch in profiles/hbm_traffic.json, tied to the
SHA-256 of the kernel's source so that a later change to the kernel makes
the entry stale (reported as null).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np
import torch

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

from paper_2105_11004_amd import api  # noqa: E402
from paper_2105_11004_amd import workloads as W  # noqa: E402

CSRC = ROOT / "paper_2105_11004_amd" / "csrc"
TRAFFIC_FILE = ROOT / "profiles" / "hbm_traffic.json"
COPY_BYTES = 1 << 30
DEFAULT_WORKLOAD = "dense_bf16_4Mx1024"
# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


def _src_hash(path: Path) -> str:
    return hashlib.sha256(path.read_bytes()).hexdigest()[:16]


def make_workload(name: str, device):
    cfg = dict(W.CONFIGS[name])
    idx = list(W.CONFIGS).index(name) + 1
    if name.endswith("_exact"):
        A = W.dense_gaussian(cfg["n"], cfg["d"], W.data_seed(idx), dtype=torch.float32, device=device)
    elif name.startswith("dense_f32"):
        heavy = 0.0 if name.endswith("_bwd") else 0.01  # the backward workload has no heavy rows
        A = W.low_rank_coherent(cfg["n"], cfg["d"], cfg["rank"], W.data_seed(idx), heavy_frac=heavy, device=device)
    elif name.startswith("dense_f64"):
        A = W.dense_gaussian(cfg["n"], cfg["d"], W.data_seed(idx), dtype=torch.float64, device=device)
    elif name.startswith("dense_bf16"):
        A = W.row_scaled_bf16(cfg["n"], cfg["d"], W.data_seed(idx), device=device)
    elif name.startswith("csr_f32"):
        A = W.sparse_power_law(cfg["n"], cfg["d"], cfg["zero_cols"], W.data_seed(idx), device=device)
    else:
        raise SystemExit(f"unknown workload {name}")
    return A, cfg, W.sketch_seed(idx)


def _is_csr(A) -> bool:
    return not isinstance(A, torch.Tensor)


def _n(A) -> int:
    return A.n if _is_csr(A) else A.shape[0]


def _values(A):
    return A.values if _is_csr(A) else A


def resolve_precision(A, precision: str) -> str:
    """'auto': the FP32-level form for BF16 storage (Z in three BF16 parts),
    the native form otherwise."""
    if precision != "auto":
        return precision
    return "bf16x3" if (not _is_csr(A) and A.dtype == torch.bfloat16) else "native"


def a_bytes(A) -> int:
    """Bytes of A as stored (dense: n*d elements; CSR: row_ptr, col_idx, values)."""
    if _is_csr(A):
        return A.row_ptr.numel() * 8 + A.col_idx.numel() * 4 + A.values.numel() * A.values.element_size()
    return A.shape[0] * A.shape[1] * A.element_size()


# kernels that carry each pass (for the traffic counters and the profiles)
def pass_kernels_for(csr: bool, dtype: torch.dtype, precision: str, d: int = 0) -> dict:
    if csr:
        # FP32 Z whose d rows (64 floats each) fit in 152 KiB of LDS: the
        # 16-lane group kernel; else the one-row-per-wave kernel
        grp = dtype != torch.float64 and d * 64 * 4 <= 152 * 1024
        return {"pass1_countsketch": ("countsketch_csr_kernel", CSRC / "sketch.hip"),
                "pass2_rownorm": ("rownorm_csr_grp_kernel" if grp else "rownorm_csr_kernel",
                                  CSRC / "rownorm_csr.hip")}
    if precision == "fp32" or dtype == torch.float64:
        p2 = ("rownorm_dense_kernel", CSRC / "rownorm.hip")
    elif dtype == torch.bfloat16:
        p2 = ("rownorm_bf16s_kernel", CSRC / "rownorm_bf16.hip")
    else:
        p2 = ("rownorm_x3_kernel", CSRC / "rownorm.hip")
    return {"pass1_countsketch": ("countsketch_dense_kernel", CSRC / "sketch.hip"), "pass2_rownorm": p2}


def pass_kernels(A, precision: str) -> dict:
    return pass_kernels_for(_is_csr(A), _values(A).dtype, precision, A.d if _is_csr(A) else A.shape[1])


def expected_rank(cfg) -> int:
    return min(cfg["d"] - cfg.get("zero_cols", 0), cfg.get("rank", cfg["d"]))


def phase_work(A, cfg, mode: str = "jl", sketch: str = "gauss") -> dict:
    """Algorithmic work of each phase of one estimate: bytes for the passes
    over A (HBM-bound), FP64 flops for the n-independent phases (their
    dominant kernels are FP64 MFMA GEMMs and the pivoting that drives them).
    Without the JL step and for the exact scores, Z has d columns of which
    the first r are live: pass 2 reads A once per live tile of 64 columns;
    the exact scores' Gram pass (dense: 2 n d^2 flops on the FP64 matrix
    cores; CSR: one read of A at least) falls in the form_z phase."""
    n, d, m, r_cs, k = _n(A), cfg["d"], cfg["m"], cfg["r_cs"], cfg["k"]
    theta_es = 8 if _values(A).dtype == torch.float64 else 4
    r = expected_rank(cfg)
    out = _phase_work_mode(A, cfg, mode, n, d, m, r_cs, k, theta_es, r)
    if (sketch == "gauss" and not _is_csr(A) and A.dtype == torch.bfloat16 and r_cs % 8 == 0
            and out["gaussian_transform"][1] > 0):
        # BF16-stored dense A: the transform runs as six products of
        # three-part BF16 splits on the BF16 matrix cores (FP32-level
        # arithmetic), so it is priced by those products against that peak;
        # pass 1 then writes G_m as three BF16 parts (6 bytes an entry) and
        # S A as FP32 (the split starts from its FP32 value)
        out["gaussian_transform"] = ("mfma_bf16", 6 * 2.0 * m * r_cs * d)
        if mode == "jl":
            out["pass1_countsketch"] = ("hbm", a_bytes(A) + 4 * r_cs * d + 8 * d * k + 6 * m * r_cs)
        else:  # no G_k
            out["pass1_countsketch"] = ("hbm", a_bytes(A) + 4 * r_cs * d + 6 * m * r_cs)
    if sketch == "srht":
        # no G_m: pass 1 writes S A (and G_k); the SRHT reads S A once and
        # writes A~ at least (its radix passes add the in-place round trips)
        out["pass1_countsketch"] = ("hbm", a_bytes(A) + 8 * (r_cs * d + (d * k if mode == "jl" else 0)))
        out["gaussian_transform"] = ("hbm", 8 * (r_cs * d + m * d))
    return out


def _phase_work_mode(A, cfg, mode, n, d, m, r_cs, k, theta_es, r) -> dict:
    if mode == "qless":
        # Algorithm 6: no sketch; one pass over A for the norms and one per
        # step (min(k, r) steps, the last one stopping at the cutoff)
        steps = min(k, r)
        tiles = -(-steps // 64)
        return {
            "pass1_countsketch": ("hbm", 0),
            "gaussian_transform": ("hbm", 0),
            "rank_revealing_qr": ("hbm", (steps + 1) * a_bytes(A)),
            "form_z": ("mfma_fp64", float(steps) * steps * d),
            "pass2_rownorm": ("hbm", tiles * (a_bytes(A) + n * theta_es)),
        }
    if mode != "jl":
        tiles = -(-r // 64)
        if mode == "exact":
            gram = ("hbm", a_bytes(A)) if _is_csr(A) else ("mfma_fp64", 2.0 * n * d * d)
        else:
            gram = ("mfma_fp64", float(r) * r * d)
        return {
            "pass1_countsketch": ("hbm", a_bytes(A) + 8 * (r_cs * d + m * r_cs)),
            "gaussian_transform": ("mfma_fp64", 2.0 * m * r_cs * d),
            "rank_revealing_qr": ("mfma_fp64", 2.0 * m * d * d + d ** 3 / 3.0),
            "form_z": gram,
            "pass2_rownorm": ("hbm", tiles * (a_bytes(A) + n * theta_es)),
        }
    return {
        # pass 1 reads A once and writes S A (FP64) plus the two Gaussian
        # matrices it draws on the side (G_m m x r_cs, G_k d x k, FP64)
        "pass1_countsketch": ("hbm", a_bytes(A) + 8 * (r_cs * d + m * r_cs + d * k)),
        # A~ = G_m (S A): 2 m r_cs d flops
        "gaussian_transform": ("mfma_fp64", 2.0 * m * r_cs * d),
        # Gram 2 m d^2 + pivoted Cholesky d^3 / 3 (to the rank r: r d^2 - ...)
        "rank_revealing_qr": ("mfma_fp64", 2.0 * m * d * d + d ** 3 / 3.0),
        # Z = R11^{-1} G_k: r^2 k flops
        "form_z": ("mfma_fp64", float(r) * r * k),
        # pass 2 reads A once and writes theta~
        "pass2_rownorm": ("hbm", a_bytes(A) + n * theta_es),
    }


def rooflines(A, cfg, phases_ms: dict, traffic: dict, mode: str = "jl", sketch: str = "gauss") -> dict:
    out = {}
    for name, (bound, work) in phase_work(A, cfg, mode, sketch).items():
        t = phases_ms[name] * 1e-3
        if work == 0:
            continue  # a phase this mode does not have
        if bound == "hbm":
            ach = work / t / 1e9
            out[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": traffic.get(name), "algorithmic_bytes": work}
        else:
            ach = work / t / 1e12
            peak, dt = (BF16_PEAK_TFLOPS, "bf16") if bound == "mfma_bf16" else (FP64_PEAK_TFLOPS, "f64")
            out[name] = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                         "frac": ach / peak, "traffic": None, "algorithmic_flops": work, "dtype": dt}
    return out


# ---------------------------------------------------------------------------- CPU oracle
def _host_rows(A, lo: int, hi: int) -> np.ndarray:
    """Rows lo..hi-1 of dense A as FP64 numpy (exact for BF16/FP32)."""
    return A[lo:hi].to(torch.float64).cpu().numpy()


def cpu_baseline(A, cfg, seed, target_s: float = 10.0, mode: str = "jl", sketch: str = "gauss"):
    """Times the oracle's estimator on the first n_s rows of the workload
    (same d, sketch sizes and seed), growing n_s until about a quarter of
    target_s; when that covers the whole workload, the whole workload is
    timed repeatedly until about target_s and the mean is reported."""
    from oracle import leverage as L

    def oracle(Ah):
        if mode == "qless":
            return L.ls_qless_qr(Ah, cfg["zeta"], cfg["k"])
        if mode == "exact":
            return L.ls_hrn_exact(Ah, seed, cfg["r_cs"], cfg["m"], cfg["zeta"], sketch=sketch)
        o = L.ls_hrn_approx(Ah, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], sketch=sketch)
        if mode == "nojl":
            return L.theta_prime(Ah, o.perm[:o.rank], o.R11)
        return o

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    n = _n(A)
    ns = min(n, 1 << 15)
    S = A.to_scipy() if _is_csr(A) else None

    def host(rows):
        return S[:rows] if S is not None else _host_rows(A, 0, rows)

    while True:
        Ah = host(ns)
        t0 = time.perf_counter()
        oracle(Ah)
        dt = time.perf_counter() - t0
        if dt > target_s / 4 or ns >= n:
            break
        ns = min(n, ns * max(2, int(target_s / 4 / max(dt, 1e-3))))
    reps, total = 1, dt
    while ns >= n and total < target_s:
        t0 = time.perf_counter()
        oracle(Ah)
        total += time.perf_counter() - t0
        reps += 1
    dt = total / reps
    what = f"first {ns} rows of the workload" if ns < n else f"the whole workload ({n} rows), mean of {reps} runs"
    return {"value": ns / dt, "unit": "rows/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{what}, full estimator ({ORACLE_STEPS[mode]}), "
                      f"FP64 NumPy/SciPy, {dt:.2f} s per run"}


ORACLE_STEPS = {"jl": "sketch, QRCP, Z, row norms", "nojl": "sketch, QRCP, R11^-1, row norms",
                "exact": "sketch, QRCP, Gram of A_K, eigh, row norms",
                "qless": "Q-less pivoted QR of A, R^-1, row norms"}


def _stats(ratio: np.ndarray) -> dict:
    return {"median": float(np.median(ratio)), "q01": float(np.quantile(ratio, 0.01)),
            "q99": float(np.quantile(ratio, 0.99)),
            "frac_within_0.5": float(np.mean(np.abs(ratio - 1.0) <= 0.5))}


def accuracy_report(A, cfg, seed, forms: dict, n_rows: int = 2000, mode: str = "jl", sketch: str = "gauss") -> dict:
    """theta~ of each form (name -> full theta~ on the device) on sampled
    rows against (i) the oracle's FP64 estimator with the same sketch (the
    JL estimate, or theta' without the JL step; for the exact scores the
    exact scores themselves) and (ii) the exact scores (Algorithm 5's Gram
    route over the whole matrix, streamed in row blocks, cutoff zeta); raw
    and sum-normalised (theta~ * r / sum theta~, which uses sum theta =
    rank)."""
    from oracle import leverage as L

    n = _n(A)
    rows = np.sort(np.random.default_rng(12345).choice(n, min(n_rows, n), replace=False))
    t0 = time.perf_counter()
    if _is_csr(A):
        Ah = A.to_scipy()
        o = L.ls_hrn_approx(Ah, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], rows=rows, sketch=sketch)
        blk = 1 << 20
        chunks = lambda: ((lo, Ah[lo:lo + blk].toarray()) for lo in range(0, n, blk))  # noqa: E731
    else:
        Ah = A.float().cpu().numpy() if A.dtype == torch.bfloat16 else A.cpu().numpy()
        o = L.ls_hrn_approx(Ah, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], rows=rows, sketch=sketch)
        blk = 1 << 16
        chunks = lambda: ((lo, Ah[lo:lo + blk]) for lo in range(0, n, blk))  # noqa: E731
    t_same = time.perf_counter() - t0
    t0 = time.perf_counter()
    exact, rho = L.theta_gram_rows(chunks, rows, max(cfg["zeta"], 1e-6))
    t_exact = time.perf_counter() - t0
    if mode == "nojl":
        same = L.theta_prime(Ah, o.perm[:o.rank], o.R11, rows=rows)
    elif mode == "qless":
        same, _ = L.ls_qless_qr(Ah, cfg["zeta"], cfg["k"], rows=rows)
    elif mode == "exact":
        same = exact  # the exact scores of A_K are those of A when r = rank(A)
    else:
        same = o.theta_rows
    del Ah
    out = {"rows_sampled": int(rows.size), "oracle_rank": int(o.rank), "exact_rank": int(rho),
           "oracle_s": {"same_sketch": t_same, "exact_gram": t_exact}, "mode": mode, "forms": {}}
    for name, theta in forms.items():
        th = theta.to(torch.float64)
        total = float(th.sum().item())
        got = th.cpu().numpy()[rows]
        rel = np.abs(got - same) / np.maximum(np.abs(same), 1e-300)
        rel = rel[np.abs(same) > 0] if mode != "jl" else rel
        live = exact > 1e-300
        ratio = got[live] / exact[live]
        norm = ratio * (o.rank / total) if total > 0 else ratio
        out["forms"][name] = {
            "vs_oracle_same_sketch": {"max_rel": float(rel.max()), "p99_rel": float(np.quantile(rel, 0.99))},
            "vs_exact_theta": {"raw": _stats(ratio), "normalised": _stats(norm)},
            "sum_theta": total, "rank": int(o.rank),
        }
    return out


# ---------------------------------------------------------------------------- traffic
def traffic_for(workload: str, A, precision: str) -> dict:
    """Counter bytes per launch of each pass for this workload, or None when
    the counters predate the kernel's current source."""
    out = {}
    if not TRAFFIC_FILE.exists():
        return out
    data = json.loads(TRAFFIC_FILE.read_text()).get(workload, {})
    for key, (kernel, src) in pass_kernels(A, precision).items():
        ent = data.get(key)
        ok = ent and ent.get("kernel") == kernel and ent.get("source_sha") == _src_hash(src) \
            and ent.get("precision") == precision
        out[key] = ent.get("bytes_per_launch") if ok else None
    return out


def traffic_run(workload: str, precision: str):
    dev = torch.device("cuda:0")
    api.load_library()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # the calibration copy: COPY_BYTES read, COPY_BYTES written
    torch.cuda.synchronize()
    del src, dst
    A, cfg, seed = make_workload(workload, dev)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"],
                            precision=resolve_precision(A, precision))
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    print("traffic run done", flush=True)


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f)), files[0]


def _per_dispatch(rows, counter: str):
    """[(kernel name, KiB)] in dispatch order (values summed over the
    counter's instances within a dispatch)."""
    acc: dict = {}
    order = []
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        if key not in acc:
            acc[key] = [r.get("Kernel_Name", ""), 0.0]
            order.append(key)
        acc[key][1] += float(r["Counter_Value"])
    return [tuple(acc[k]) for k in order]


def traffic_summarize(fetch_dir: str, write_dir: str, workload: str, precision: str):
    cfg = W.CONFIGS[workload]
    fetch_rows, fetch_file = _counter_rows(fetch_dir)
    write_rows, write_file = _counter_rows(write_dir)
    fetch = _per_dispatch(fetch_rows, "FETCH_SIZE")
    write = _per_dispatch(write_rows, "WRITE_SIZE")

    def copy_kib(disp):
        cands = [v for name, v in disp if "copy" in name.lower()]
        if not cands:
            raise SystemExit("calibration copy kernel not found in the counter output")
        return max(cands)  # the 1 GiB copy is the largest copy dispatch

    f_read = COPY_BYTES / (copy_kib(fetch) * 1024.0)
    f_write = COPY_BYTES / (copy_kib(write) * 1024.0)
    dtype = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[cfg["dtype"]]
    csr = workload.startswith("csr")
    if precision == "auto":
        precision = "bf16x3" if (dtype == torch.bfloat16 and not csr) else "native"
    kern = pass_kernels_for(csr, dtype, precision, cfg["d"])
    # the algorithmic bytes of the passes, from the workload itself (a CSR
    # matrix's are those of its row_ptr, col_idx and values)
    A, _, _ = make_workload(workload, torch.device("cuda:0") if torch.cuda.is_available() else torch.device("cpu"))
    algorithmic = {k: w for k, (b, w) in phase_work(A, cfg).items() if b == "hbm"}
    del A
    entry = {"copy_bytes": COPY_BYTES, "factor_read": f_read, "factor_write": f_write}
    lines = [f"# HBM traffic per launch, workload {workload}, precision {precision} "
             f"(rocprofv3 FETCH_SIZE / WRITE_SIZE, KiB per dispatch)",
             f"# fetch counters: {fetch_file}", f"# write counters: {write_file}",
             f"# calibration: 1 GiB device copy counted {copy_kib(fetch):.0f} KiB fetched, "
             f"{copy_kib(write):.0f} KiB written -> factors read {f_read:.4f}, write {f_write:.4f}"]
    for key, (pattern, src) in kern.items():
        fk = [v for name, v in fetch if pattern in name]
        wk = [v for name, v in write if pattern in name]
        if not fk or not wk:
            continue
        fb = fk[-1] * 1024.0 * f_read
        wb = wk[-1] * 1024.0 * f_write
        entry[key] = {"kernel": pattern, "precision": precision, "source_sha": _src_hash(src),
                      "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                      "algorithmic_bytes": algorithmic.get(key), "launches_seen": len(fk)}
        alg = algorithmic.get(key)
        ratio = f" (ratio {(fb + wb) / alg:.3f})" if alg else ""
        lines.append(f"{key} ({pattern}): fetch {fb / 1e9:.4f} GB + write {wb / 1e9:.4f} GB = "
                     f"{(fb + wb) / 1e9:.4f} GB per launch; algorithmic "
                     f"{(alg or 0) / 1e9:.4f} GB{ratio}; kernel source sha {entry[key]['source_sha']}")
    data = json.loads(TRAFFIC_FILE.read_text()) if TRAFFIC_FILE.exists() else {}
    data = {k: v for k, v in data.items() if isinstance(v, dict) and k in W.CONFIGS}
    data[workload] = entry
    TRAFFIC_FILE.parent.mkdir(exist_ok=True)
    TRAFFIC_FILE.write_text(json.dumps(data, indent=1) + "\n")
    print("\n".join(lines))


# ---------------------------------------------------------------------------- the benchmark
def read_ceiling(A, stream, reps: int = 5) -> dict:
    """GB/s of liblev's plain streaming read (16-byte loads, no arithmetic
    but a checksum) over the workload's largest device buffer (dense: A;
    CSR: the values), timed with events on the stream it runs on: the read
    bandwidth a pass over A could reach at best."""
    buf = _values(A)
    nbytes = buf.numel() * buf.element_size() // 16 * 16
    sink = api.lev_debug_stream_read(buf, nbytes, stream=stream)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(reps):
        api.lev_debug_stream_read(buf, nbytes, sink, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return {"GB/s": nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes, "ms": ms, "kernel": "stream_read_kernel",
            "frac_of_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def time_steps(plan, bwd, steps: int, stream) -> float:
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        plan.run()
        if bwd is not None:
            bwd.run()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def phase_times(plan, bwd, steps: int, stream):
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(api.LEV_PHASES)] for _ in range(steps)]
    for row in ev:
        for e in row:
            e.record(stream)
    torch.cuda.synchronize()
    bwd_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    for s in range(steps):
        api.lev_set_phase_events(ev[s])
        plan.run()
        if bwd is not None:
            bwd_ev[s][0].record(stream)
            bwd.run()
            bwd_ev[s][1].record(stream)
    torch.cuda.synchronize()
    api.lev_set_phase_events(None)
    phases, spread = {}, {}
    for i, name in enumerate(api.PHASE_NAMES):
        vals = [ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(steps)]
        phases[name] = float(np.mean(vals))
        spread[name] = {"median": float(np.median(vals)), "min": float(np.min(vals)), "max": float(np.max(vals))}
    step_vals = [ev[s][0].elapsed_time(ev[s][len(api.PHASE_NAMES)]) for s in range(steps)]
    spread["step"] = {"median": float(np.median(step_vals)), "min": float(np.min(step_vals)),
                      "max": float(np.max(step_vals))}
    bms = float(np.mean([e[0].elapsed_time(e[1]) for e in bwd_ev])) if bwd is not None else None
    return phases, spread, bms


ALGORITHMS = {"jl": "LS-HRN-approx (Algorithm 10)", "exact": "LS-HRN-exact (Algorithm 7)",
              "nojl": "Algorithm 10 without the JL step (Pi_2 = I)",
              "qless": "exact scores via a Q-less pivoted QR (Algorithm 6)"}
SKETCH_NAMES = {"gauss": "CountGauss G (S A) (Algorithm 3)", "srht": "SRHT F (S A) (Section 4)"}


def precondition_report(steps: int) -> dict:
    """Section 6's experiment on the GPU: kappa(A N) for the 50,000 x 60
    matrices with singular values linspace(1, r, 60), r = 1e-2 ... 1e-10,
    N from Algorithm 11 (SVD) and from the pivoted QR, 20 sketches each
    (m = 2d, r_cs = 5 (d^2 + d)); then the time of the preconditioner and of
    LSQR on A N (40 steps) there and on a 2^20 x 256 FP32 Gaussian."""
    dev = torch.device("cuda:0")
    n, d = 50000, 60
    r_cs, m = 5 * (d * d + d), 2 * d
    out = {"shape": [n, d], "r_cs": r_cs, "m": m, "zeta": 1e-10, "runs": 20, "kappa": {}}
    for e in range(2, 11):
        r = 10.0 ** -e
        A = W.fixed_spectrum(n, np.linspace(1.0, r, d), 100 + e)
        Ah = A.numpy()
        Ag = A.to(dev)
        row = {"kappa_A": float(np.linalg.cond(Ah))}
        for method in ("svd", "qr"):
            ks = []
            for seed in range(20):
                N, k = api.lev_precondition(Ag, seed, r_cs, m, 1e-10, method)
                kk = int(k.item())
                ks.append(float(np.linalg.cond(Ah @ N.cpu().numpy()[:, :kk])))
            row[method] = {"min": min(ks), "mean": float(np.mean(ks)), "max": max(ks)}
        out["kappa"][f"{r:.0e}"] = row
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps

    timing = {}
    for name, A in (("50000x60_f64_r1e-6", W.fixed_spectrum(n, np.linspace(1.0, 1e-6, d), 7).to(dev)),
                    ("1Mx256_f32_gaussian", W.dense_gaussian(1 << 20, 256, 8, dtype=torch.float32, device=dev))):
        nn, dd = A.shape
        rc, mm = (r_cs, m) if dd == d else (4096, 512)
        b = torch.randn(nn, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(9))
        N, _ = api.lev_precondition(A, 1, rc, mm, 1e-10, "qr")
        t_pre = timed(lambda: api.lev_precondition(A, 1, rc, mm, 1e-10, "qr"), max(2, steps // 4))
        t_ls = timed(lambda: api.lev_lsqr(A, N, b, 40), max(2, steps // 4))
        x, hist = api.lev_lsqr(A, N, b, 40)
        per_step = t_ls / 40
        if dd <= 128:
            t_svd = timed(lambda: api.lev_precondition(A, 1, rc, mm, 1e-10, "svd"), max(2, steps // 4))
        else:
            t_svd = None
        timing[name] = {"precondition_ms": t_pre, "precondition_svd_ms": t_svd,
                        "lsqr_40_steps_ms": t_ls, "lsqr_ms_per_step": per_step,
                        "lsqr_hbm_gbs": 2 * A.numel() * A.element_size() / (per_step * 1e-3) / 1e9,
                        "residual_estimate_first_last": [float(hist[0]), float(hist[-1])]}
    out["timing"] = timing
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--precision", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--mode", choices=("jl", "exact", "nojl", "qless"), default="jl",
                    help="jl: Algorithm 10; exact: Algorithm 7 (LS-HRN-exact); nojl: Algorithm 10 without "
                         "the JL step (Pi_2 = I); qless: Algorithm 6 (Q-less pivoted QR of A, k = step cap)")
    ap.add_argument("--exact", action="store_true", help="same as --mode exact")
    ap.add_argument("--sketch", choices=("gauss", "srht"), default="gauss",
                    help="gauss: A~ = G (S A) (Algorithm 3); srht: A~ = F (S A), the SRHT composition of Section 4")
    ap.add_argument("--precondition", action="store_true",
                    help="run Section 6's preconditioning experiment and LSQR timing instead of the estimator")
    ap.add_argument("--traffic-run", action="store_true", help="the process a counter run profiles")
    ap.add_argument("--traffic-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    args = ap.parse_args()
    if args.exact:
        args.mode = "exact"
    if args.traffic_summarize:
        traffic_summarize(*args.traffic_summarize, args.workload, args.precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the row-sharded multi-GPU design is described, not built)"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.traffic_run:
        traffic_run(args.workload, args.precision)
        return
    if args.precondition:
        api.load_library()
        print(json.dumps({"report": "preconditioning (Section 6, Algorithm 11) and LSQR on A N",
                          **precondition_report(args.steps)}), flush=True)
        return
    dev = torch.device("cuda:0")
    api.load_library()
    print(f"# generating workload {args.workload}", file=sys.stderr, flush=True)
    A, cfg, seed = make_workload(args.workload, dev)
    precision = resolve_precision(A, args.precision)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], precision=precision,
                            mode=args.mode, sketch=args.sketch)
    bwd = None
    if args.workload.endswith("_bwd"):
        bwd = api.BackwardPlan(plan, torch.rand(A.shape[0], device=dev, dtype=A.dtype,
                                                generator=torch.Generator(device=dev).manual_seed(5)))
    for _ in range(args.warmup):
        plan.run()
        if bwd is not None:
            bwd.run()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)

    # the headline: K steps with no instrumentation inside them; then the
    # breakdown from K more steps with liblev's phase events
    ms = time_steps(plan, bwd, args.steps, stream)
    phases, spread, bms = phase_times(plan, bwd, args.steps, stream)
    n = _n(A)
    traffic = traffic_for(args.workload, A, precision)
    roofs = rooflines(A, cfg, phases, traffic, args.mode, args.sketch)
    # the headline roofline is the dominant kernel's: the longest of the
    # phases that one kernel launch carries (the passes over A); the slowest
    # phase overall is reported beside it (the rank-revealing step is a chain
    # of d dependent pivot steps over ~70 launches, bound by the latency of a
    # step rather than by a throughput roofline)
    kern = pass_kernels(A, precision)
    single = [k for k in ("pass1_countsketch", "pass2_rownorm") if k in roofs and args.mode == "jl"]
    dom = max(single or list(roofs), key=lambda k: phases[k])
    headline = dict(roofs[dom])
    headline["phase"] = dom
    headline["kernel"] = kern[dom][0] if dom in kern else None
    slowest = max(roofs, key=lambda k: phases[k])
    slow = {"phase": slowest, "ms": phases[slowest], "share_of_step": phases[slowest] / ms,
            "roofline": roofs[slowest]}
    if slowest == "rank_revealing_qr":
        slow["per_pivot_us"] = phases[slowest] * 1e3 / expected_rank(cfg)
    out = {
        "metric": "rows/sec and HBM GB/s for rSLS estimate at eps=0.5 (fraction of HBM roofline)",
        "value": n / (ms * 1e-3),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"float32": "f32", "float64": "f64", "bfloat16": "bf16"}[str(_values(A).dtype).split(".")[1]],
        "data": "synthetic (seeded, generated on the GPU)",
        "config": {"workload": args.workload, "n": n, "d": cfg["d"], "r_cs": cfg["r_cs"], "m": cfg["m"],
                   "k": cfg["k"], "zeta": cfg["zeta"], "precision": precision,
                   "algorithm": ALGORITHMS[args.mode], "sketch": SKETCH_NAMES[args.sketch]},
        "roofline": headline,
        "slowest_phase": slow,
        "rooflines": roofs,
        "phases_ms": phases,
        "phases_ms_spread": spread,
    }
    # the measured ceiling: a plain streaming read of A's largest buffer
    ceil = read_ceiling(A, stream)
    out["read_ceiling"] = ceil
    if headline.get("unit") == "GB/s":
        headline["frac_of_read_ceiling"] = headline["achieved"] / ceil["GB/s"]
    if "pass1_countsketch" in roofs:
        out["passes_hbm_frac"] = {
            "pass1": roofs["pass1_countsketch"]["frac"], "pass2": roofs["pass2_rownorm"]["frac"],
            "both": (roofs["pass1_countsketch"]["algorithmic_bytes"] + roofs["pass2_rownorm"]["algorithmic_bytes"])
            / ((phases["pass1_countsketch"] + phases["pass2_rownorm"]) * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if bwd is not None:
        out["backward_ms"] = bms
        out["backward_hbm_gbs"] = 3 * a_bytes(A) / (bms * 1e-3) / 1e9  # two reads of A, one write of the gradient
    forms = {precision: plan.theta.clone()}
    if args.mode == "jl" and not _is_csr(A) and A.dtype == torch.bfloat16:
        # the other BF16 forms on the same GPU: time and theta~
        out["bf16_forms"] = {precision: {"ms_per_step": ms, "pass2_ms": phases["pass2_rownorm"]}}
        for other in ("bf16", "bf16x2", "bf16x3"):
            if other == precision:
                continue
            p2 = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], precision=other,
                                  sketch=args.sketch)
            p2.run()
            t = time_steps(p2, None, max(3, args.steps // 4), stream)
            ph, _, _ = phase_times(p2, None, max(3, args.steps // 4), stream)
            out["bf16_forms"][other] = {"ms_per_step": t, "pass2_ms": ph["pass2_rownorm"]}
            forms[other] = p2.theta.clone()
            del p2
    if not args.no_accuracy:
        print("# accuracy on sampled rows (oracle: same sketch, and exact scores)", file=sys.stderr, flush=True)
        out["accuracy"] = accuracy_report(A, cfg, seed, forms, mode=args.mode, sketch=args.sketch)
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, cfg, seed, mode=args.mode, sketch=args.sketch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
