"""HBM traffic of the two passes over A, from rocprofv3 hardware counters.

Two counter runs, each in a process of its own (the profiler collects one
counter set per run), then a summary:

    rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o fetch -- python3 -m paper_2105_11004_amd.hbm_traffic run
    rocprofv3 --pmc WRITE_SIZE -d OUT/write -o write -- python3 -m paper_2105_11004_amd.hbm_traffic run
    python3 -m paper_2105_11004_amd.hbm_traffic summarize OUT/fetch OUT/write [--workload NAME]

``run`` first copies a 1 GiB device buffer to another (a plain copy kernel
that reads and writes exactly 1 GiB), then runs lev_estimate twice on the
benchmark workload.  ``summarize`` reads the per-dispatch counter values
(KiB), scales each counter by what it read for the copy (known bytes over
counted bytes: the calibration factor), and writes profiles/hbm_traffic.json
(bytes per launch for each pass, tied to the SHA-256 of the kernel's source
so that a later change to the kernel invalidates it) and a text summary.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
COPY_BYTES = 1 << 30
KERNELS = {
    # the benchmark's FP32 pass runs the BF16x3 kernel (rownorm_x3_kernel);
    # the other dense forms run rownorm_dense_kernel
    "pass2_rownorm": ("rownorm_x3_kernel", PKG / "csrc" / "rownorm.hip"),
    "pass1_countsketch": ("countsketch_dense_kernel", PKG / "csrc" / "sketch.hip"),
}


def src_hash(path: Path) -> str:
    return hashlib.sha256(path.read_bytes()).hexdigest()[:16]


def run(workload: str):
    import torch

    sys.path.insert(0, str(ROOT))
    from bench import make_workload  # the benchmark's own input recipe
    from paper_2105_11004_amd import api

    dev = torch.device("cuda:0")
    api.load_library()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # the calibration copy: COPY_BYTES read, COPY_BYTES written
    torch.cuda.synchronize()
    del src, dst
    A, cfg, seed = make_workload(workload, dev)
    plan = api.EstimatePlan(A, seed, cfg["r_cs"], cfg["m"], cfg["k"], cfg["zeta"])
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    print("hbm_traffic run done", flush=True)


def _rows(d: str):
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


def summarize(fetch_dir: str, write_dir: str, workload: str):
    sys.path.insert(0, str(ROOT))
    from paper_2105_11004_amd import workloads as W

    cfg = W.CONFIGS[workload]
    fetch_rows, fetch_file = _rows(fetch_dir)
    write_rows, write_file = _rows(write_dir)
    fetch = _per_dispatch(fetch_rows, "FETCH_SIZE")
    write = _per_dispatch(write_rows, "WRITE_SIZE")

    def copy_kib(disp):
        cands = [v for name, v in disp if "copy" in name.lower()]
        if not cands:
            raise SystemExit("calibration copy kernel not found in the counter output")
        return max(cands)  # the 1 GiB copy is the largest copy dispatch

    f_read = COPY_BYTES / (copy_kib(fetch) * 1024.0)
    f_write = COPY_BYTES / (copy_kib(write) * 1024.0)
    es = {"f32": 4, "f64": 8, "bf16": 2}[cfg["dtype"]]
    n, d = cfg["n"], cfg["d"]
    algorithmic = {"pass2_rownorm": n * d * es + n * (8 if cfg["dtype"] == "f64" else 4),
                   "pass1_countsketch": n * d * es + cfg["r_cs"] * d * 8}
    out = {"workload": workload, "copy_bytes": COPY_BYTES, "factor_read": f_read, "factor_write": f_write}
    lines = [f"# HBM traffic per launch, workload {workload} (rocprofv3 FETCH_SIZE / WRITE_SIZE, KiB per dispatch)",
             f"# fetch counters: {fetch_file}", f"# write counters: {write_file}",
             f"# calibration: 1 GiB device copy counted {copy_kib(fetch):.0f} KiB fetched, "
             f"{copy_kib(write):.0f} KiB written -> factors read {f_read:.4f}, write {f_write:.4f}"]
    for key, (pattern, src) in KERNELS.items():
        fk = [v for name, v in fetch if pattern in name]
        wk = [v for name, v in write if pattern in name]
        if not fk or not wk:
            continue
        fb = fk[-1] * 1024.0 * f_read
        wb = wk[-1] * 1024.0 * f_write
        out[key] = {"source_sha": src_hash(src), "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                    "algorithmic_bytes": algorithmic[key], "launches_seen": len(fk)}
        lines.append(f"{key}: fetch {fb / 1e9:.4f} GB + write {wb / 1e9:.4f} GB = {(fb + wb) / 1e9:.4f} GB per launch; "
                     f"algorithmic {algorithmic[key] / 1e9:.4f} GB (ratio {(fb + wb) / algorithmic[key]:.3f}); "
                     f"kernel source sha {out[key]['source_sha']}")
    (ROOT / "profiles").mkdir(exist_ok=True)
    (ROOT / "profiles" / "hbm_traffic.json").write_text(json.dumps(out, indent=1) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="dense_f32_1Mx256_rank128")
    s = sub.add_parser("summarize")
    s.add_argument("fetch_dir")
    s.add_argument("write_dir")
    s.add_argument("--workload", default="dense_f32_1Mx256_rank128")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload)
    else:
        summarize(a.fetch_dir, a.write_dir, a.workload)


if __name__ == "__main__":
    main()
