"""Autotuner for the TSQR launch geometry (leaf height and tree arity).

    python -m paper_1402_6964_amd.tune --m 10000000 --n 25 [--dtype f32] [--layout row] [--leaf f32] [--pad 0]
    python -m paper_1402_6964_amd.tune --batched

For one input shape it times tsnmf_tsqr_r_ex over a grid of leaf heights
(rows per slab, the TSQR leaf) and, for n <= 32, tree group sizes (slab
factors merged per tree node) with HIP events.  It rejects any configuration
whose R differs from the default configuration's by more than the rounding
bound of the precision used (every configuration computes the same R up to
rounding), and records the fastest in the text table
paper_1402_6964_amd/tuned.txt, keyed like the library's table by (input
dtype, layout, row-block precision, contiguous rows, n, floor(log2 m)).
tsnmf_tune_load(path) makes the library apply it to every tsnmf_tsqr_r call
that matches an entry; tsnmf.tsqr_r(X, config="tuned") applies the entry for
X explicitly.

The row-block height (rows one wave holds in registers per Householder pass)
is a compile-time constant per width, chosen by measurement; the tunable
"leaf height" of the TSQR is the slab, which is a runtime parameter.

--batched tunes the batched call on the 512-matrix workload: the slab height
of each width class (16 and 32 columns, one wave per slab; up to 64; up to
128) as a power-of-two multiple of its default, one class at a time (each
class keeps the best value found for it while the next is swept).  Every
configuration's R factors must equal the default's within the rounding bound;
the best goes into the table's "batch" line, which tsnmf_tune_load makes the
library apply to every tsnmf_tsqr_r_batched call.
"""

import argparse
import math
import os

import torch

from . import synth, tsnmf

TUNED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.txt")
HEADER = ("# tsnmf autotune table: tsqr <dtype> <layout> <leaf precision> <ld == n> <n> <floor(log2 m)> "
          "<leaf_rows> <tree_arity> <wy_panel>\n"
          "#                       batch <slab shift, 16 columns> <32 columns> <up to 64> <up to 128>\n")
BATCH = ("batch",)


def key(dtype, layout, leaf, ldeq, n, m):
    return (dtype, layout, leaf, int(bool(ldeq)), int(n), int(math.log2(max(m, 1))))


def load(path=None):
    """The table as {key: (leaf_rows, tree_arity, wy_panel, comment)}, and the
    batched call's slab shifts as {BATCH: (shifts, comment)}."""
    out = {}
    try:
        with open(path or TUNED) as f:
            for line in f:
                body, _, note = line.partition("#")
                p = body.split()
                if len(p) == 5 and p[0] == "batch":
                    out[BATCH] = (tuple(int(v) for v in p[1:]), note.strip())
                    continue
                if len(p) not in (9, 10) or p[0] != "tsqr":
                    continue
                k = (p[1], p[2], p[3], int(p[4]), int(p[5]), int(p[6]))
                out[k] = (int(p[7]), int(p[8]), int(p[9]) if len(p) == 10 else 0, note.strip())
    except OSError:
        pass
    return out


def save(table, path=None):
    with open(path or TUNED, "w") as f:
        f.write(HEADER)
        if BATCH in table:
            shifts, note = table[BATCH]
            f.write("batch " + " ".join(str(int(v)) for v in shifts) + (f"  # {note}" if note else "") + "\n")
        for k in sorted(k for k in table if k != BATCH):
            leaf_rows, arity, wy, note = table[k]
            f.write(f"tsqr {k[0]} {k[1]} {k[2]} {k[3]} {k[4]} {k[5]} {leaf_rows} {arity} {wy}"
                    + (f"  # {note}" if note else "") + "\n")


def key_of(X, leaf_f64=False):
    m, n = X.shape
    lay, ld = tsnmf._layout(X)
    dt = {torch.float32: "f32", torch.float64: "f64"}[X.dtype]
    col = lay == tsnmf.COL_MAJOR
    leaf = "f64" if (dt == "f64" or leaf_f64) else "f32"
    return key(dt, "col" if col else "row", leaf, ld == (m if col else n), n, m)


def lookup(X, leaf_f64=False, path=None):
    e = load(path).get(key_of(X, leaf_f64))
    if e is None:
        return None
    return tsnmf.TsqrConfig(leaf_rows=e[0], tree_arity=e[1], rows_per_lane=0, wy_panel=e[2])


def time_config(X, cfg, leaf_f64=False, reps=20):
    m, n = X.shape
    lay, ld = tsnmf._layout(X)
    flags = tsnmf._DTYPE_FLAG[X.dtype] | lay | (tsnmf.LEAF_F64 if leaf_f64 else 0)
    Rbuf = torch.empty((n, n), dtype=torch.float64, device=X.device)
    cs = torch.empty(n, dtype=torch.float64, device=X.device)
    for _ in range(3):
        tsnmf._check("tsnmf_tsqr_r_ex", tsnmf.tsnmf_tsqr_r_ex(X, m, n, ld, flags, Rbuf, cs, cfg))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        tsnmf.tsnmf_tsqr_r_ex(X, m, n, ld, flags, Rbuf, cs, cfg)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps, Rbuf.t().cpu()


def leaf_grid(m):
    """Leaf heights around the default's: slabs for 512 .. 4096 leaves, and the
    fixed heights 256, 512 and 1024 rows (lengthened by the library where the
    leaf count would exceed its ticket area)."""
    return [0] + sorted({max(64, m // p) for p in (512, 1024, 1536, 2048, 3072, 4096)} | {256, 512, 1024})


def tune(X, leaf_f64=False, grid=None, arity_grid=None, wy_grid=None, verbose=True):
    m, n = X.shape
    t0, R0 = time_config(X, None, leaf_f64)
    tol = 1e-5 if (X.dtype == torch.float32 and not leaf_f64) else 1e-11
    grid = leaf_grid(m) if grid is None else grid
    if arity_grid is None:
        arity_grid = [0, 8, 12, 16, 20, 24, 32] if n <= 32 else [0]
    if wy_grid is None:      # blocked (16-column panels) or unblocked trailing update
        wy_grid = [16, 1] if (X.dtype == torch.float32 and not leaf_f64 and 33 <= n <= 64) else [0]
    best = (t0, 0, 0, 0)
    results = [{"leaf_rows": 0, "tree_arity": 0, "wy_panel": 0, "ms": t0}]
    for leaf in grid:
        for ar in arity_grid:
            for wy in wy_grid:
                if leaf == 0 and ar == 0 and wy in (0, 16):
                    continue
                cfg = tsnmf.TsqrConfig(leaf_rows=int(leaf), tree_arity=int(ar), rows_per_lane=0, wy_panel=int(wy))
                ms, R = time_config(X, cfg, leaf_f64)
                err = float((R - R0).abs().max() / R0.abs().max())
                ok = err <= tol
                results.append({"leaf_rows": int(leaf), "tree_arity": int(ar), "wy_panel": int(wy), "ms": ms,
                                "err": err, "ok": ok})
                if verbose:
                    print(f"leaf_rows {leaf:9d} arity {ar:3d} wy {wy:2d}  {ms:8.3f} ms  "
                          f"{m * n * X.element_size() / ms / 1e6:8.1f} GB/s  err {err:.1e}", flush=True)
                if ok and ms < best[0]:
                    best = (ms, int(leaf), int(ar), int(wy))
    note = f"{best[0]:.4f} ms against {t0:.4f} ms default"
    return key_of(X, leaf_f64), (best[1], best[2], best[3], note), results


def time_batch(b, cfg, reps=5):
    b.run(config=cfg)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.run(config=cfg)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps, [r.clone() for r, _ in b.results()]


def tune_batched(b, verbose=True, grid=(0, 1, 2, 3)):
    """Per-class slab shifts of the batched call, one class at a time."""
    best = [0, 0, 0, 0]
    t0, R0 = time_batch(b, tsnmf.batch_config(best))
    tbest = t0
    for c in range(4):
        for v in grid:
            if v == best[c]:
                continue
            cand = list(best)
            cand[c] = v
            ms, R = time_batch(b, tsnmf.batch_config(cand))
            err = max(float((r - r0).abs().max() / r0.abs().max().clamp_min(1e-300)) for r, r0 in zip(R, R0))
            ok = err <= 1e-5
            if verbose:
                print(f"shifts {cand}  {ms:8.3f} ms  err {err:.1e}{'' if ok else '  REJECTED'}", flush=True)
            if ok and ms < tbest:
                tbest, best = ms, cand
    return tuple(best), f"{tbest:.3f} ms against {t0:.3f} ms default"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batched", action="store_true", help="tune the batched call on the 512-matrix workload")
    ap.add_argument("--m", type=int, default=10_000_000)
    ap.add_argument("--n", type=int, default=25)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--layout", choices=["row", "col"], default="row")
    ap.add_argument("--leaf", choices=["f32", "f64"], default="f32")
    ap.add_argument("--pad", type=int, default=0, help="extra elements of the row stride (row-major)")
    ap.add_argument("--no-save", action="store_true")
    args = ap.parse_args()
    if args.batched:
        shapes = synth.batch_shapes()
        mats = [synth.batch_matrix(q, m, n, device="cuda")["X"] for q, (m, n) in enumerate(shapes)]
        b = tsnmf.Batch(mats)
        shifts, note = tune_batched(b)
        print("batch", shifts, note)
        if not args.no_save:
            table = load()
            table[BATCH] = (shifts, note)
            save(table)
        return
    dt = torch.float32 if args.dtype == "f32" else torch.float64
    if args.layout == "row":
        X = synth.random_matrix(args.m, args.n + args.pad, device="cuda", dtype=dt, seed_tag=11)[:, :args.n]
    else:
        X = synth.random_matrix(args.n, args.m, device="cuda", dtype=dt, seed_tag=11).t()
    k, best, _ = tune(X, leaf_f64=args.leaf == "f64")
    print(k, best)
    if not args.no_save:
        table = load()
        table[k] = best
        save(table)


if __name__ == "__main__":
    main()
