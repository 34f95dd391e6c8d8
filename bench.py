"""Benchmark: one fused MCL iteration (expansion + prune/select/recover +
inflation + change) on the 1,000,000-vertex planted-cluster graph (~100
nnz/column, 50,000 power-law clusters, 5% inter-cluster edges, seed 1001),
on one MI355X.

Prints ONE JSON line:
  value      = expansion GFLOP/s (multiply-adds of A*A per second of the
               whole fused step, inputs resident in HBM)
  roofline   = the dominant kernel (the table bin with the largest time):
               algorithmic bytes per launch / its HIP-event time, vs 8 TB/s
  cpu_baseline = the CPU oracle on a bounded random sample of columns
Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "expansion GFLOP/s + output nnz/s at n=1M; speedup learned/batched vs plain"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the fused iteration kernel, per bin:
#   12 B per multiply-add (row index + value of every gathered A_*k entry)
#   28 B per nonzero of B_*j (colptr pair of A_*k + own row index and value)
#   12 B per output entry written, 8 B per column (count)
BYTES_PER_FLOP, BYTES_PER_BNZ, BYTES_PER_OUT, BYTES_PER_COL = 12, 28, 12, 8


COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_numeric_lds_cfg1.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2002_10083_amd", "csrc", "spgemm.hip")


def measured_traffic(kernel_key):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy), or None when
    the summary is missing, is for another kernel, or the kernel source has
    changed since it was taken."""
    import hashlib
    try:
        kv = dict(l.strip().split("=", 1) for l in open(TRAFFIC_FILE) if "=" in l and not l.startswith("#"))
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if kv.get("source_sha256") != sha or kv.get("kernel_key") != kernel_key:
        return None
    return int(float(kv["hbm_bytes_per_launch"]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bin_bytes(st, b):
    return (BYTES_PER_FLOP * st["bin_flops"][b] + BYTES_PER_BNZ * st["bin_bnnz"][b]
            + BYTES_PER_OUT * st["bin_out"][b] + BYTES_PER_COL * st["bin_cols"][b])


def cpu_baseline(W, target_s=12.0, seed=7):
    """The CPU oracle (expand + prune + inflate) on a random sample of columns."""
    import numpy as np
    import oracle
    A = oracle.normalize(W)
    rng = np.random.default_rng(seed)
    n = A.ncols

    def run(frac):
        cols = np.sort(rng.choice(n, size=max(1, int(frac * n)), replace=False))
        Bs = A.restrict_columns(cols)
        t = time.perf_counter()
        C, flops, nnz = oracle.expand(A, Bs)
        P, _ = oracle.prune(C)
        oracle.inflate(P, 2.0)
        return time.perf_counter() - t, int(flops.sum()), int(nnz.sum()), len(cols)

    dt, fl, nz, k = run(0.002)
    frac = min(1.0, 0.002 * target_s / max(dt, 1e-3))
    dt, fl, nz, k = run(frac)
    return {"value": round(fl / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d of %d columns (uniform, seed %d): expand+prune+inflate, %.1f s, "
                      "%.3g multiply-adds, %.3g product nnz/s"
                      % (k, n, seed, dt, fl, nz / dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--estimator", default="cohen", choices=["cohen", "bound"])
    ap.add_argument("--policy", type=lambda x: int(x, 0), default=None,
                    help="bin launch policy (default: tuned table if present)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from mclgen import config1_graph
    from paper_2002_10083_amd import mcl, tuning

    torch.cuda.set_device(0)
    t0 = time.time()
    W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
    log("generated n=%d nnz=%d in %.1f s" % (W.ncols, W.nnz, time.time() - t0))
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)
    torch.cuda.synchronize()
    est = mcl.EST_COHEN if args.estimator == "cohen" else mcl.EST_BOUND
    policy, scale, keys = tuning.load_policy("iterate")
    if args.policy is not None:
        policy = args.policy
    params = mcl.default_params(estimator=est, bin_policy=policy, est_scale=scale, cohen_keys=keys)

    if args.calibrate_copy:
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        G, _, st = mcl.iterate(A, params)
        del G
    torch.cuda.synchronize()
    sts = []
    t = time.perf_counter()
    for i in range(args.steps):
        G, change, st = mcl.iterate(A, params)
        sts.append(st)
        del G
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ms_step = dt / args.steps * 1e3
    flops = sts[0]["flops"]
    nnz_prod = sts[0]["nnz_product"]
    kept = sts[0]["nnz_kept"]
    gflops = flops * args.steps / dt / 1e9

    # dominant kernel: the bin with the largest mean time over the timed steps
    nb = 8
    mean_ms = [float(np.mean([s["bin_ms"][b] for s in sts])) for b in range(nb)]
    dom = int(np.argmax(mean_ms))
    byt = bin_bytes(sts[0], dom)
    achieved = byt / (mean_ms[dom] * 1e-3) / 1e9
    name = ("k_numeric_lds<%d slots>" % (128 << dom)) if dom < 7 else "k_numeric_global"
    variant = (policy >> (4 * dom)) & 15 if dom < 7 else 0
    kernel_key = "bin%d-v%d-keys%d" % (dom, variant, keys)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel_key),
            "kernel": name, "kernel_key": kernel_key,
            "kernel_ms": round(mean_ms[dom], 3), "algorithmic_bytes": int(byt)}
    total_bytes = sum(bin_bytes(sts[0], b) for b in range(nb))
    numeric_ms = float(np.mean([s["t_numeric_ms"] for s in sts]))

    out = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "one fused MCL iteration (expand+prune/select/recover+inflate) on a "
                               "planted-cluster graph, n=%d, ~100 nnz/col, seed 1001" % W.ncols,
                   "n": W.ncols, "nnz": W.nnz, "flops": flops, "estimator": args.estimator,
                   "bin_policy": hex(policy), "est_scale": scale, "cohen_keys": keys,
                   "prune": "theta=1e-4 S=1100 R=1400 pct=0.9 r=2"},
        "output_nnz_per_s": round(nnz_prod * args.steps / dt, 1),
        "kept_nnz_per_s": round(kept * args.steps / dt, 1),
        "nnz_product": nnz_prod, "nnz_kept": kept,
        "n_overflow": sts[0]["n_overflow"], "n_global": sts[0]["n_global"],
        "phase_ms": {k: round(float(np.mean([s[k] for s in sts])), 3) for k in
                     ("t_symbolic_ms", "t_estimate_ms", "t_numeric_ms", "t_fallback_ms",
                      "t_compact_ms", "t_total_ms")},
        "numeric_phase_GBps": round(total_bytes / (numeric_ms * 1e-3) / 1e9, 1),
        "roofline": roof,
    }
    log("bins ms:", [round(x, 2) for x in mean_ms])
    if not args.no_cpu_baseline:
        t1 = time.time()
        out["cpu_baseline"] = cpu_baseline(W)
        log("cpu baseline took %.1f s" % (time.time() - t1))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
