#!/usr/bin/env python3
"""Throughput of the single-pass TSQR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]

A step is one tsnmf_tsqr_r call on the flow-cytometry-shaped workload
(10,000,000 x 25 FP32 row-major, 1.0 GB, synthetic near-separable data resident
in HBM): row-block Householder leaves with fused l1 column sums, the FP64
reduction tree and the finalisation of R.  `value` is GB/s of X (bytes of X
divided by the mean step time).  The line also carries:
  roofline      the leaf kernel's algorithmic bytes per launch (every
                element of X once) over its mean duration, timed with HIP
                events recorded by the library on the launch stream during the
                timed steps, against 8 TB/s of HBM; `traffic` is the measured
                HBM bytes per launch from the committed rocprofv3 counter
                summary when it was taken on the current leaf source; its FP32
                flops (2 m n^2) against the vector peaks ride along (`alu`);
  cpu_baseline  the CPU oracle (plain FP64 numpy Householder TSQR) timed on
                this host: over all of X on up to 16 worker processes (the
                host's CPU count is recorded), and on one thread over a
                bounded row sample;
  r_error       ||R^T R - X^T X||_F / ||X||_F^2 and the column-norm error of
                the benchmarked R against the oracle's reference sums of X;
  extras        the other hot-path workloads, each timed after the main steps
                (skipped with --no-extras): the batched TSQR of 512 uneven
                matrices (one graph-captured persistent launch, against one
                FP64 tsnmf_tsqr_r call per matrix), the heat-transfer-shaped
                50,000,000 x 64 column-major matrix, the 20,000,000 x 128
                Gaussian projection (BF16 matrix cores and FP32 vector units,
                and its generator alone), the 100,000 x 20 FP64 example, and
                the one-pass path over 64 MiB row blocks from device, pinned
                and pageable host memory (host rates include the copies).
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
FP32_VECTOR_PEAK = 157.3    # FP32 vector/matrix peak of MI355X (256 CUs x 2.4 GHz, packed FP32)
FP32_UNPACKED_PEAK = 78.6   # FP32 FMA on the vector ALUs without packed instructions (all HIP code here is compiled without them)
METRIC = "TSQR GB/s of X (fraction of HBM peak) + batched matrices/s at fixed R error"
WORKLOAD = {"workload": "flow_cytometry", "m": 10_000_000, "n": 25, "dtype_in": "fp32",
            "layout": "row-major", "bytes": 10_000_000 * 25 * 4, "r": 16}
LEAF_KERNEL = "tsqr_small_kernel<float, float, 25, 6, 1>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tsqr_leaf_flow_cytometry.md")
TUNED_FILE = os.path.join(ROOT, "paper_1402_6964_amd", "tuned.txt")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and R check")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU oracle time")
    ap.add_argument("--no-extras", action="store_true", help="time only the main workload")
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


def cpu_baseline(X_gpu, R_gpu, cs_gpu, target_s, pool):
    """Oracle timed on the host: on all worker cores over the whole input, and
    on one thread over a bounded sample; R error of the benchmarked R."""
    import numpy as np
    import threadpoolctl
    from oracle import parallel as opar
    from oracle import tsqr as otsqr

    out = {}
    m, n = X_gpu.shape
    X = X_gpu.cpu().numpy()
    all_cores = None
    if pool is not None:
        pool.load(X)
        t0 = time.perf_counter()
        pool.tsqr_r(1000)
        t_all = time.perf_counter() - t0
        all_cores = {"value": m * n * 4 / t_all / 1e9, "unit": "GB/s", "cores": pool.workers,
                     "kind": "oracle",
                     "sample": f"all {m} x {n} FP32 rows, FP64 numpy Householder leaves of 1000 rows + binary "
                               f"tree (aligned runs of leaves in {pool.workers} worker processes, the top of "
                               f"the tree in the parent; the same R bit for bit), {t_all:.1f} s"}
        pool.close()
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
    single = {
        "value": rows * n * 4 / t / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
        "sample": f"first {rows} rows of the {m} x {n} FP32 input, FP64 numpy Householder leaves "
                  f"of 1000 rows + binary tree, {t:.1f} s, one thread"}
    if all_cores is not None:
        out["cpu_baseline"] = {**all_cores, "host_cores": opar.host_cores(), "single_thread": single}
    else:
        out["cpu_baseline"] = {**single, "host_cores": opar.host_cores()}
    # R error of the benchmarked R against the oracle's reference sums of all of X
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


def geometry(tuned, dt, lay, leaf, ldeq, n, m):
    """The launch geometry tsnmf_tsqr_r uses for this key: the tuned entry, or
    the library default."""
    import math
    if tuned:
        e = tuned.get((dt, lay, leaf, ldeq, n, int(math.log2(max(m, 1)))))
        if e is not None:
            return {"source": "tuned.txt", "leaf_rows": e[0], "tree_arity": e[1], "wy_panel": e[2],
                    "note": e[3]}
    return {"source": "library default"}


def _note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _gram_error(R, X64):
    import numpy as np
    G = X64.T @ X64
    return float(np.linalg.norm(R.T @ R - G) / np.trace(G))


def extras(torch, tsnmf, synth, dev, check=True, tuned=None):
    """The other hot-path workloads, a few timed repetitions each."""
    import numpy as np
    out = {}

    # batched TSQR: 512 matrices, m log-uniform in [1e4, 2e6], n in {16, 32, 64, 128}
    _note("batched: generating 512 matrices")
    shapes = synth.batch_shapes()
    mats = [synth.batch_matrix(q, m, n, device=dev)["X"] for q, (m, n) in enumerate(shapes)]
    total_bytes = sum(m * n * 4 for m, n in shapes)
    flops = sum(2.0 * m * n * n for m, n in shapes)
    b = tsnmf.Batch(mats)
    b.run()                                        # sizes the workspace outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    g.replay()
    t_batch = _timed(torch, g.replay, 5)
    _note(f"batched: {t_batch * 1e3:.2f} ms per batch; timing the per-matrix FP64 baseline")
    # baseline: one FP64 tsnmf_tsqr_r call (leaf kernel + tree kernel) per matrix
    Rs = [torch.empty((n, n), dtype=torch.float64, device=dev) for _, n in shapes]
    css = [torch.empty(n, dtype=torch.float64, device=dev) for _, n in shapes]
    stream = torch.cuda.current_stream(dev)
    flags = tsnmf.F32 | tsnmf.LEAF_F64

    def per_matrix():
        for X, R, c in zip(mats, Rs, css):
            st = tsnmf.tsnmf_tsqr_r(X, X.shape[0], X.shape[1], X.shape[1], flags, R, c, stream)
            if st != 0:
                raise tsnmf.TsnmfError("tsnmf_tsqr_r", st)

    per_matrix()
    t_base = _timed(torch, per_matrix, 2)
    _note(f"batched: baseline {t_base * 1e3:.2f} ms per batch")
    res = b.results()
    # R error on one matrix per width (the shortest), against the FP64 reference sums
    errs, agree = [], []
    if check:
        for n in (16, 32, 64, 128):
            q = min((i for i, s in enumerate(shapes) if s[1] == n), key=lambda i: shapes[i][0])
            X64 = mats[q].cpu().numpy().astype(np.float64)
            Rb = res[q][0].cpu().numpy()
            errs.append(_gram_error(Rb, X64))
            Rf = tsnmf.colmajor_square(Rs[q]).cpu().numpy()
            agree.append(float(np.abs(Rb - Rf).max() / np.abs(Rf).max()))
    out["batched"] = {
        "workload": "512 FP32 row-major matrices, m log-uniform in [1e4, 2e6], n in {16, 32, 64, 128}",
        "matrices": len(shapes), "bytes": total_bytes, "flops": flops,
        "ms_per_batch": round(t_batch * 1e3, 3),
        "matrices_per_s": round(len(shapes) / t_batch, 1),
        "gbs": round(total_bytes / t_batch / 1e9, 1),
        "tflops_fp32": round(flops / t_batch / 1e12, 2),
        "baseline_fp64_per_matrix_ms_per_batch": round(t_base * 1e3, 3),
        "baseline_matrices_per_s": round(len(shapes) / t_base, 1),
        "speedup_vs_baseline": round(t_base / t_batch, 2),
        "gram_rel_max": max(errs) if errs else None, "gram_tol": 1e-6,
        "max_rel_diff_vs_fp64_baseline": max(agree) if agree else None,
        "graph_captured": True,
        "geometry": ({"source": "tuned.txt", "slab_shift": list(tuned[("batch",)][0]), "note": tuned[("batch",)][1]}
                     if tuned and ("batch",) in tuned else {"source": "library default"}),
    }
    del mats, b, g, Rs, css, res
    torch.cuda.empty_cache()

    # heat-transfer-shaped matrix, column-major (ld = m)
    _note("heat transfer: generating 50,000,000 x 64")
    d = synth.heat_transfer(device=dev)
    X = d["X"]
    m, n = X.shape
    R = torch.empty((n, n), dtype=torch.float64, device=dev)
    c = torch.empty(n, dtype=torch.float64, device=dev)

    def heat():
        st = tsnmf.tsnmf_tsqr_r(X, m, n, m, tsnmf.F32 | tsnmf.COL_MAJOR, R, c, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_tsqr_r", st)

    hb = m * n * 4
    hflops = 2.0 * m * n * n
    out["heat_transfer"] = {"workload": "50,000,000 x 64 FP32 column-major (12.8 GB)",
                            "geometry": geometry(tuned, "f32", "col", "f32", 1, n, m)}
    # the library's choice (tsnmf_tsqr_r), and the blocked compact-WY and
    # unblocked leaves side by side (tsnmf_tsqr_r_ex)
    for name, cfg in (("default", None),
                      ("wy16", tsnmf.TsqrConfig(leaf_rows=0, tree_arity=0, rows_per_lane=0, wy_panel=16)),
                      ("unblocked", tsnmf.TsqrConfig(leaf_rows=0, tree_arity=0, rows_per_lane=0, wy_panel=1))):
        def heat():
            if cfg is None:
                st = tsnmf.tsnmf_tsqr_r(X, m, n, m, tsnmf.F32 | tsnmf.COL_MAJOR, R, c, stream)
            else:
                st = tsnmf.tsnmf_tsqr_r_ex(X, m, n, m, tsnmf.F32 | tsnmf.COL_MAJOR, R, c, cfg, stream)
            if st != 0:
                raise tsnmf.TsnmfError("tsnmf_tsqr_r", st)

        heat()
        tsnmf.tsnmf_profile_query(0)
        tsnmf.tsnmf_profile_enable(2)
        t = _timed(torch, heat, 5)
        tsnmf.tsnmf_profile_enable(0)
        _, lms, lcalls = tsnmf.tsnmf_profile_query(0)
        tsnmf.tsnmf_profile_query(1)
        lavg = lms / max(lcalls, 1) * 1e-3
        out["heat_transfer"][name] = {"ms": round(t * 1e3, 3), "gbs": round(hb / t / 1e9, 1),
                                      "leaf_ms": round(lavg * 1e3, 3), "leaf_gbs": round(hb / lavg / 1e9, 1),
                                      "leaf_tflops": round(hflops / lavg / 1e12, 1),
                                      "leaf_frac_fp32": round(hflops / lavg / 1e12 / FP32_VECTOR_PEAK, 4)}
    del X, d
    torch.cuda.empty_cache()

    # Gaussian projection Y = G^T X, k = 512
    _note("projection: generating 20,000,000 x 128")
    d = synth.projection(device=dev)
    X = d["X"]
    Xb = X.to(torch.bfloat16)
    m, n = X.shape
    k = 512
    Y = torch.empty((n, k), dtype=torch.float32, device=dev)
    proj = {}
    for name, Xin, fl, peak in (("bf16_mfma", Xb, tsnmf.BF16 | tsnmf.GP_MFMA_BF16, 2500.0),
                                ("fp32_simd", X, tsnmf.F32 | tsnmf.GP_SIMD_F32, 157.3)):
        def gp():
            st = tsnmf.tsnmf_gauss_proj(Xin, m, n, n, fl, k, 14026964, 0, Y, None, stream)
            if st != 0:
                raise tsnmf.TsnmfError("tsnmf_gauss_proj", st)
        gp()
        t = _timed(torch, gp, 3)
        tf = 2.0 * m * n * k / t / 1e12
        proj[name] = {"ms": round(t * 1e3, 3), "tflops": round(tf, 1), "peak_tflops": peak,
                      "frac": round(tf / peak, 4), "gbs": round(Xin.numel() * Xin.element_size() / t / 1e9, 1),
                      "gnormals_per_s": round(m * k / t / 1e9, 1)}
    # the generator alone on the matrix-core kernel's launch shape (G^T 1, no X
    # read): the ceiling of the BF16 path, whose MFMA work is 2 n = 256 flops
    # per normal
    sbuf = torch.empty(k, dtype=torch.float32, device=dev)

    def gen():
        st = tsnmf.tsnmf_gauss_colsum(m, k, 14026964, 0, sbuf, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_gauss_colsum", st)
    gen()
    tsnmf.tsnmf_profile_query(0)
    tsnmf.tsnmf_profile_enable(2)
    t = _timed(torch, gen, 3)
    tsnmf.tsnmf_profile_enable(0)
    _, gms, gcalls = tsnmf.tsnmf_profile_query(0)
    gker = gms / max(gcalls, 1) * 1e-3
    rng = {"ms": round(t * 1e3, 3), "kernel_ms": round(gker * 1e3, 3),
           "gnormals_per_s": round(m * k / gker / 1e9, 1)}
    proj["bf16_mfma"]["frac_of_generator_ceiling"] = round(gker * 1e3 / proj["bf16_mfma"]["ms"], 4)
    out["projection"] = {"workload": "20,000,000 x 128, k = 512", "gaussians": m * k, **proj,
                         "generator_alone": rng}
    del X, Xb, d, Y
    torch.cuda.empty_cache()

    # the 100,000 x 20 FP64 example (whole path in FP64)
    d = synth.plain_fp64(device=dev)
    X = d["X"]
    m, n = X.shape
    R = torch.empty((n, n), dtype=torch.float64, device=dev)

    def small():
        st = tsnmf.tsnmf_tsqr_r(X, m, n, n, tsnmf.F64, R, None, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_tsqr_r", st)

    small()
    t = _timed(torch, small, 20)
    # the whole example on the GPU: TSQR with 1,000-row leaves and a binary
    # tree, SPA on R D^{-1} (r = 10), NNLS for H and the residual, stream
    # ordered with no host synchronisation, then the same captured in a graph
    r = d["r"]
    cs1 = torch.empty(n, dtype=torch.float64, device=dev)
    K = torch.empty(r, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    H = torch.empty((n, r), dtype=torch.float64, device=dev)
    rel = torch.empty(1, dtype=torch.float64, device=dev)
    cfg1 = tsnmf.TsqrConfig(leaf_rows=1000, tree_arity=2, rows_per_lane=0, wy_panel=0)

    def pipeline(s=stream):
        for st in (tsnmf.tsnmf_tsqr_r_ex(X, m, n, n, tsnmf.F64, R, cs1, cfg1, s),
                   tsnmf.tsnmf_select_spa(R, n, n, n, cs1, r, K, None, info, s),
                   tsnmf.tsnmf_nnls(R, n, n, n, K, r, H, r, None, None, s),
                   tsnmf.tsnmf_residual(R, n, n, n, K, r, H, r, rel, s)):
            if st != 0:
                raise tsnmf.TsnmfError("pipeline", st)

    pipeline()
    tp = _timed(torch, pipeline, 20)
    gs = torch.cuda.Stream()
    torch.cuda.synchronize()
    gp_ = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gp_, stream=gs):
        pipeline(gs.cuda_stream)
    gp_.replay()
    tg = _timed(torch, gp_.replay, 20)
    # the other n x n selections on the same R: greedy XRAY (r picks, an NNLS
    # fit after each) and the residual curve of SPA's picks for ranks 1..r
    Kx = torch.empty(r, dtype=torch.int32, device=dev)
    infx = torch.empty(1, dtype=torch.int32, device=dev)
    Ks = torch.empty(r, dtype=torch.int32, device=dev)
    Hs = torch.empty((n, r), dtype=torch.float64, device=dev)
    curve = torch.empty(r, dtype=torch.float64, device=dev)
    infs = torch.empty(1, dtype=torch.int32, device=dev)

    def xray():
        st = tsnmf.tsnmf_select_xray(R, n, n, n, r, Kx, infx, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_select_xray", st)

    def sweep():
        st = tsnmf.tsnmf_rank_sweep(R, n, n, n, cs1, r, Ks, Hs, r, curve, infs, stream)
        if st != 0:
            raise tsnmf.TsnmfError("tsnmf_rank_sweep", st)

    xray()
    sweep()
    tx = _timed(torch, xray, 20)
    tsw = _timed(torch, sweep, 20)
    out["plain_fp64"] = {"workload": "100,000 x 20 FP64 row-major", "tsqr_ms": round(t * 1e3, 4),
                         "tsqr_gbs": round(m * n * 8 / t / 1e9, 1),
                         "pipeline": "TSQR (1,000-row leaves, binary tree) -> SPA (r = 10) -> NNLS -> residual",
                         "pipeline_us": round(tp * 1e6, 1), "pipeline_graph_us": round(tg * 1e6, 1),
                         "K": sorted(K.cpu().tolist()), "K_planted": d["K"], "residual": float(rel.item()),
                         "xray_us": round(tx * 1e6, 1), "K_xray": sorted(Kx.cpu().tolist()),
                         "rank_sweep_us": round(tsw * 1e6, 1),
                         "residual_curve": [float("%.4g" % v) for v in curve.cpu().tolist()]}
    del X, d
    torch.cuda.empty_cache()

    # One pass over row blocks (tsnmf_onepass_*), the path for matrices larger
    # than the device: the flow-cytometry matrix pushed from device memory in
    # the 64 MiB blocks the host path uses, and from pinned and pageable host
    # memory (the host rates include the host-to-device copies), with and
    # without G^T X (k = 32, matrix cores) in the same pass.
    _note("one pass: flow cytometry in 64 MiB blocks, device and host input")
    dfc = synth.flow_cytometry(device=dev)
    Xd = dfc["X"]
    m, n = Xd.shape
    Xp = Xd.cpu().pin_memory()
    Xn = Xd.cpu().numpy()
    op_out = {"workload": "flow_cytometry 10,000,000 x 25 FP32 row-major (1.0 GB), 64 MiB blocks"}

    def one_pass(kind, k):
        op = tsnmf.OnePass(n, k=k, seed=14026964, mode=tsnmf.GP_MFMA_BF16 if k else None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "device":
            br = op.block_rows
            for a in range(0, m, br):
                op.push(Xd[a:min(m, a + br)])
        else:
            op.push_host(Xp if kind == "pinned_host" else Xn)
        op.result()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        op.close()
        return t

    for kind, k in (("device", 0), ("pinned_host", 0), ("pageable_host", 0), ("device", 32), ("pinned_host", 32)):
        one_pass(kind, k)
        t = min(one_pass(kind, k) for _ in range(3))
        op_out[f"{kind}_k{k}"] = {"s": round(t, 4), "gbs": round(m * n * 4 / t / 1e9, 2)}
    out["one_pass"] = op_out
    del Xd, Xp, Xn, dfc
    torch.cuda.empty_cache()
    return out


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    # the all-core oracle's worker processes start before this process
    # touches the GPU (spawned, they never do); the box grants one GPU's share
    # of its CPUs, 16
    pool = None
    if not args.no_cpu and not args.copy_reference:
        from oracle import parallel as opar
        pool = opar.OraclePool(max(1, min(16, opar.host_cores())))
    import torch
    from paper_1402_6964_amd import synth, tsnmf

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # the committed autotune table: tsnmf_tsqr_r applies its matching entries
    tuned = None
    if os.path.exists(TUNED_FILE):
        if tsnmf.tsnmf_tune_load(TUNED_FILE) != 0:
            raise RuntimeError(f"cannot load {TUNED_FILE}")
        from paper_1402_6964_amd import tune as _tune
        tuned = _tune.load(TUNED_FILE)
    if args.copy_reference:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)        # a vector-memory kernel, not a DMA copy
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": a.numel() * 4, "launches": 5}))
        return

    wl = WORKLOAD
    _note("main: generating 10,000,000 x 25")
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
    # timed region: the library records two HIP events per call on the launch
    # stream, around the leaf kernel only (the least intrusive mode)
    tsnmf.tsnmf_profile_enable(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tsnmf.tsnmf_profile_enable(0)
    _, leaf_ms, leaf_calls = tsnmf.tsnmf_profile_query(0)
    # the reduction tree's time, from a short separate pass with every stage timed
    tsnmf.tsnmf_profile_enable(1)
    for _ in range(min(args.steps, 20)):
        step()
    torch.cuda.synchronize()
    tsnmf.tsnmf_profile_enable(0)
    tsnmf.tsnmf_profile_query(0)
    _, tail_ms, tail_calls = tsnmf.tsnmf_profile_query(1)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gbs = wl["bytes"] / (ms_per_step * 1e-3) / 1e9
    leaf_avg_ms = leaf_ms / max(leaf_calls, 1)
    achieved = wl["bytes"] / (leaf_avg_ms * 1e-3) / 1e9
    leaf_flops = 2 * wl["m"] * wl["n"] * wl["n"]          # 2 m n^2, the Householder work of the leaves
    leaf_tflops = leaf_flops / (leaf_avg_ms * 1e-3) / 1e12
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
        "config": {**wl, "workload": "flow_cytometry 10,000,000 x 25 FP32 row-major (1.0 GB), "
                                     "FP32 Householder leaves + FP64 tree",
                   "geometry": geometry(tuned, "f32", "row", "f32", 1, wl["n"], wl["m"])},
        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
        # The leaf kernel reads 4 m n bytes and does 2 m n^2 FP32 flops: 12.5
        # flop/B, below the 19.7 flop/B ridge of the 157.3 TF/s FP32 peak, so
        # its roof is HBM.  The ALU view rides along: against 157.3 TF/s, and
        # against 78.6 TF/s, the FP32 FMA rate of the vector ALUs without the
        # packed instructions that the library's kernels are compiled without.
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": LEAF_KERNEL, "kernel_avg_ms": round(leaf_avg_ms, 5),
                     "algorithmic_bytes_per_launch": wl["bytes"],
                     "algorithmic_flops_per_launch": leaf_flops,
                     "alu": {"achieved": round(leaf_tflops, 2), "unit": "TFLOP/s",
                             "peak_fp32": FP32_VECTOR_PEAK, "frac_fp32": round(leaf_tflops / FP32_VECTOR_PEAK, 4),
                             "peak_fp32_unpacked": FP32_UNPACKED_PEAK,
                             "frac_fp32_unpacked": round(leaf_tflops / FP32_UNPACKED_PEAK, 4)}},
        "tail_avg_ms": round(tail_ms / max(tail_calls, 1), 5),
    }
    _note(f"main: {ms_per_step:.4f} ms per step")
    if not args.no_cpu:
        torch.cuda.synchronize()
        _note("cpu baseline: timing the oracle")
        line.update(cpu_baseline(X, tsnmf.colmajor_square(Rbuf), cs, args.cpu_seconds, pool))
    if not args.no_extras:
        del X, d
        torch.cuda.empty_cache()
        line["extras"] = extras(torch, tsnmf, synth, dev, check=not args.no_cpu, tuned=tuned)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
