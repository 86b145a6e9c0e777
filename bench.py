#!/usr/bin/env python3
"""Throughput of the single-pass TSQR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one tsnmf_tsqr_r call on the flow-cytometry-shaped workload
(10,000,000 x 25 FP32 row-major, 1.0 GB, synthetic near-separable data resident
in HBM): row-block Householder leaves with fused l1 column sums, the FP64
reduction tree and the finalisation of R.  `value` is GB/s of X (bytes of X
divided by the mean step time).  The line also carries:
  roofline      the leaf kernel's algorithmic bytes per launch over its mean
                duration, timed with HIP events recorded by the library on the
                launch stream during the timed steps, against 8 TB/s;
  cpu_baseline  the CPU oracle (plain FP64 numpy Householder TSQR) timed on a
                bounded row sample of the same X on this host;
  r_error       ||R^T R - X^T X||_F / ||X||_F^2 and the column-norm error of
                the benchmarked R against the oracle's reference sums of X.
Only one GPU is used: --gpus above 1 exits with a message.
"""

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "TSQR GB/s of X (fraction of HBM peak) + batched matrices/s at fixed R error"
WORKLOAD = {"workload": "flow_cytometry", "m": 10_000_000, "n": 25, "dtype_in": "fp32",
            "layout": "row-major", "bytes": 10_000_000 * 25 * 4, "r": 16}
LEAF_KERNEL = "tsqr_small_kernel<float, float, 25, 6, 1>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tsqr_leaf_flow_cytometry.md")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and R check")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU oracle time")
    ap.add_argument("--copy-reference", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    return ap.parse_args()


def read_traffic():
    """Per-launch HBM bytes of the leaf kernel from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's reading)."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"^kernel_source_sha:\s*(\S+)", txt, re.M)
    t = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    if not (m and t):
        return None
    if m.group(1) != kernel_source_sha():
        return None          # kernel changed since the counters were taken
    return float(t.group(1))


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("tsqr_small.hpp", "wave.hpp", "tsqr_small_inst.hpp"):
        with open(os.path.join(ROOT, "paper_1402_6964_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(X_gpu, R_gpu, cs_gpu, target_s):
    """Oracle timed on a bounded sample; R error of the benchmarked R."""
    import numpy as np
    import threadpoolctl
    from oracle import tsqr as otsqr

    out = {}
    m, n = X_gpu.shape
    with threadpoolctl.threadpool_limits(1):
        # calibrate on a small sample, then time a sample sized for ~target_s
        rows = 20_000
        Xs = X_gpu[:rows].cpu().numpy()
        t0 = time.perf_counter()
        otsqr.tsqr_r_final(Xs, leaf_rows=1000)
        t_small = time.perf_counter() - t0
        rows = int(min(m, max(20_000, rows * target_s / max(t_small, 1e-3))))
        rows -= rows % 1000
        Xs = X_gpu[:rows].cpu().numpy()
        t0 = time.perf_counter()
        otsqr.tsqr_r_final(Xs, leaf_rows=1000)
        t = time.perf_counter() - t0
    out["cpu_baseline"] = {
        "value": rows * n * 4 / t / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
        "sample": f"first {rows} rows of the {m} x {n} FP32 input, FP64 numpy Householder leaves "
                  f"of 1000 rows + binary tree, {t:.1f} s, one thread"}
    # R error of the benchmarked R against the oracle's reference sums of all of X
    X = X_gpu.cpu().numpy()
    colsum, colsq, gram = otsqr.reference_sums(X)
    R = R_gpu.cpu().numpy()
    cs = cs_gpu.cpu().numpy()
    gerr = float(np.linalg.norm(R.T @ R - gram) / np.trace(gram))
    nerr = float(np.max(np.abs(np.linalg.norm(R, axis=0) - np.sqrt(colsq)) / np.sqrt(colsq)))
    serr = float(np.max(np.abs(cs - colsum) / colsum))
    out["r_error"] = {"gram_rel": gerr, "colnorm_rel": nerr, "colsum_rel": serr,
                      "gram_tol": 1e-6, "colnorm_tol": 1e-5,
                      "pass": bool(gerr <= 1e-6 and nerr <= 1e-5)}
    return out


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1402_6964_amd import synth, tsnmf

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_reference:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": a.numel() * 4, "launches": 5}))
        return

    wl = WORKLOAD
    d = synth.flow_cytometry(m=wl["m"], n=wl["n"], r=wl["r"], device=dev)
    X = d["X"]
    m, n = X.shape
    flags = tsnmf.F32 | tsnmf.ROW_MAJOR
    Rbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    cs = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        st = tsnmf.tsnmf_tsqr_r(X, m, n, n, flags, Rbuf, cs, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_tsqr_r", st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tsnmf.tsnmf_profile_query(0)
    tsnmf.tsnmf_profile_query(1)
    tsnmf.tsnmf_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tsnmf.tsnmf_profile_enable(False)
    _, leaf_ms, leaf_calls = tsnmf.tsnmf_profile_query(0)
    _, tail_ms, tail_calls = tsnmf.tsnmf_profile_query(1)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gbs = wl["bytes"] / (ms_per_step * 1e-3) / 1e9
    leaf_avg_ms = leaf_ms / max(leaf_calls, 1)
    achieved = wl["bytes"] / (leaf_avg_ms * 1e-3) / 1e9
    traffic = read_traffic()
    line = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "flow_cytometry 10,000,000 x 25 FP32 row-major (1.0 GB), "
                               "FP32 Householder leaves + FP64 tree", **wl},
        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": LEAF_KERNEL, "kernel_avg_ms": round(leaf_avg_ms, 5),
                     "algorithmic_bytes_per_launch": wl["bytes"]},
        "tail_avg_ms": round(tail_ms / max(tail_calls, 1), 5),
    }
    if not args.no_cpu:
        torch.cuda.synchronize()
        line.update(cpu_baseline(X, tsnmf.colmajor_square(Rbuf), cs, args.cpu_seconds))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
