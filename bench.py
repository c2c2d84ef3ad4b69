"""Benchmark of the rSLS estimator (LS-HRN-approx) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one lev_estimate call over the whole workload resident in HBM:
Gaussian draws, pass 1 (CountSketch S A), the Gaussian transform, the
rank-revealing factorisation, Z = R11^{-1} G_k and pass 2 (theta~); for the
backward workload (name ending in _bwd) also the adjoint of w^T theta~.  Prints
one JSON line with rows/s, the per-phase times, the roofline of the
dominant kernel (HBM-bound pass 2) measured live with HIP events, and the
CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = ROOT / "profiles" / "hbm_traffic.json"
KERNEL_SOURCES = {"pass2_rownorm": ROOT / "paper_2105_11004_amd" / "csrc" / "rownorm.hip",
                  "pass1_countsketch": ROOT / "paper_2105_11004_amd" / "csrc" / "sketch.hip"}


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


def a_bytes(A) -> int:
    """Bytes of A as stored (dense: n*d elements; CSR: row_ptr, col_idx, values)."""
    if _is_csr(A):
        return A.row_ptr.numel() * 8 + A.col_idx.numel() * 4 + A.values.numel() * A.values.element_size()
    return A.shape[0] * A.shape[1] * A.element_size()


def bytes_per_launch(A, cfg) -> dict:
    vals = A.values if _is_csr(A) else A
    n = A.n if _is_csr(A) else A.shape[0]
    d = cfg["d"]
    theta_es = 8 if vals.dtype == torch.float64 else 4
    return {
        # pass 2 reads A once and writes theta~ (Z is ~KB, read from cache)
        "pass2_rownorm": a_bytes(A) + n * theta_es,
        # pass 1 reads A once and writes S A (FP64)
        "pass1_countsketch": a_bytes(A) + cfg["r_cs"] * d * 8,
    }


def cpu_baseline(A, cfg, seed, target_s: float = 10.0, exact: bool = False):
    """Times the oracle's estimator on the first n_s rows of the workload
    (same d, sketch sizes and seed), growing n_s until about a quarter of
    target_s; when that covers the whole workload, the whole workload is
    timed repeatedly until about target_s and the mean is reported."""
    from oracle import leverage as L

    def oracle(Ah):
        if exact:
            return L.ls_hrn_exact(Ah, seed, cfg["r_cs"], cfg["m"], cfg["zeta"])
        return L.ls_hrn_approx(Ah, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"])

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    n = A.n if _is_csr(A) else A.shape[0]
    ns = min(n, 1 << 15)
    S = A.to_scipy() if _is_csr(A) else None

    def host(rows):
        if S is not None:
            return S[:rows]
        return A[:rows].to(torch.float64).cpu().numpy() if A.dtype == torch.bfloat16 else A[:rows].cpu().numpy()

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
            "sample": f"{what}, full estimator ({'sketch, QRCP, Gram of A_K, eigh, row norms' if exact else 'sketch, QRCP, Z, row norms'}), "
                      f"FP64 NumPy/SciPy, {dt:.2f} s per run"}


def traffic_for(kernel: str):
    if not TRAFFIC_FILE.exists():
        return None
    data = json.loads(TRAFFIC_FILE.read_text())
    ent = data.get(kernel)
    if not ent or ent.get("source_sha") != _src_hash(KERNEL_SOURCES[kernel]):
        return None  # counters predate the current kernel
    return ent.get("bytes_per_launch")


def _median_ms(fn, stream, reps=5) -> float:
    fn()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def copy_ceiling(A, stream) -> dict:
    """Measured ceilings on A's storage: a device-to-device copy (bytes read +
    bytes written) and a read-only reduction (torch's sum over its words)."""
    src = (A.values if _is_csr(A) else A).reshape(-1).view(torch.uint8)
    nbytes = src.numel()
    dst = torch.empty_like(src)
    copy_ms = _median_ms(lambda: dst.copy_(src), stream)
    del dst
    # the reduction reads the bytes as FP32 words (their values do not matter here)
    words = src[: nbytes // 4 * 4].view(torch.float32)
    read_ms = min(_median_ms(lambda: torch.sum(words), stream), _median_ms(lambda: torch.amax(words), stream))
    return {"torch_copy_gbs": 2 * nbytes / (copy_ms * 1e-3) / 1e9, "torch_read_gbs": nbytes / (read_ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense_f32_1Mx256_rank128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="native")
    ap.add_argument("--exact", action="store_true",
                    help="time Algorithm 7 (LS-HRN-exact: dense FP32/FP64, d <= 64) instead of Algorithm 10")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU row-sharded design is described, not built)"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    dev = torch.device("cuda:0")
    api.load_library()
    print(f"# generating workload {args.workload}", file=sys.stderr, flush=True)
    A, cfg, seed = make_workload(args.workload, dev)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"], precision=args.precision,
                            exact=args.exact)
    backward = args.workload.endswith("_bwd")
    if backward:
        bwd = api.BackwardPlan(plan, torch.rand(A.shape[0], device=dev, dtype=A.dtype,
                                                generator=torch.Generator(device=dev).manual_seed(5)))
    for _ in range(args.warmup):
        plan.run()
        if backward:
            bwd.run()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    # per-step phase events (created by one record each, then handed to liblev)
    stream = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(api.LEV_PHASES)] for _ in range(args.steps)]
    for row in ev:
        for e in row:
            e.record(stream)
    torch.cuda.synchronize()

    # the headline: K steps with no instrumentation inside them
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        plan.run()
        if backward:
            bwd.run()
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms = total_ms / args.steps

    # the breakdown: K more steps with liblev's phase events (recording them
    # adds a little time of its own between the kernels)
    bwd_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for s in range(args.steps):
        api.lev_set_phase_events(ev[s])
        plan.run()
        if backward:
            bwd_ev[s][0].record(stream)
            bwd.run()
            bwd_ev[s][1].record(stream)
    torch.cuda.synchronize()
    api.lev_set_phase_events(None)

    phases = {}
    spread = {}
    for i, name in enumerate(api.PHASE_NAMES):
        vals = [ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(args.steps)]
        phases[name] = float(np.mean(vals))
        spread[name] = {"median": float(np.median(vals)), "min": float(np.min(vals)), "max": float(np.max(vals))}
    step_vals = [ev[s][0].elapsed_time(ev[s][len(api.PHASE_NAMES)]) for s in range(args.steps)]
    spread["step"] = {"median": float(np.median(step_vals)), "min": float(np.min(step_vals)),
                      "max": float(np.max(step_vals))}
    copy_gbs = copy_ceiling(A, stream)
    n = A.n if _is_csr(A) else A.shape[0]
    vals = A.values if _is_csr(A) else A
    bpl = bytes_per_launch(A, cfg)
    dom = "pass2_rownorm"
    achieved = bpl[dom] / (phases[dom] * 1e-3) / 1e9
    pass1_gbs = bpl["pass1_countsketch"] / (phases["pass1_countsketch"] * 1e-3) / 1e9
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
        "dtype": {"float32": "f32", "float64": "f64", "bfloat16": "bf16"}[str(vals.dtype).split(".")[1]],
        "data": "synthetic (seeded, generated on the GPU)",
        "config": {"workload": args.workload, "n": n, "d": cfg["d"], "r_cs": cfg["r_cs"], "m": cfg["m"],
                   "k": cfg["k"], "zeta": cfg["zeta"], "precision": args.precision,
                   "algorithm": "LS-HRN-exact (Algorithm 7)" if args.exact else "LS-HRN-approx (Algorithm 10)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom), "kernel": dom},
        "phases_ms": phases,
        "phases_ms_spread": spread,
        "pass1_hbm_gbs": pass1_gbs,
        "pass1_frac": pass1_gbs / HBM_PEAK_GBS,
        # measured ceilings beside the spec-sheet peak, on the same GPU: a
        # device-to-device copy of A's bytes (read + write) and a torch
        # reduction that reads them once
        "measured_ceilings": copy_gbs,
    }
    if backward:
        bms = float(np.mean([e[0].elapsed_time(e[1]) for e in bwd_ev]))
        out["backward_ms"] = bms
        out["backward_hbm_gbs"] = 3 * a_bytes(A) / (bms * 1e-3) / 1e9  # two reads of A, one write of the gradient
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, cfg, seed, exact=args.exact)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
