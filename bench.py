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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_numeric_part_cfg1.txt")
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


def part_bytes(st, b):
    """Algorithmic bytes of the accumulation kernel of a split bin: the
    gathers and step metadata as above, plus its unsorted writes of the
    unpruned entries (12 B each)."""
    return (BYTES_PER_FLOP * st["bin_flops"][b] + BYTES_PER_BNZ * st["bin_bnnz"][b]
            + BYTES_PER_OUT * st["bin_prod"][b])


# split launch shapes (waves per part, slots per wave, parts) by (bin, variant),
# as in the library's launch table
SPLIT_SHAPES = {(3, 4): (1, 512, 2), (3, 5): (1, 512, 2), (4, 4): (2, 512, 2), (4, 5): (1, 512, 4),
                (4, 6): (1, 512, 4), (5, 5): (4, 512, 2), (5, 6): (2, 512, 4), (5, 7): (1, 512, 8),
                (6, 6): (2, 512, 8), (6, 7): (1, 512, 16), (6, 8): (4, 512, 4), (6, 9): (8, 512, 2),
                (6, 10): (2, 512, 8), (6, 11): (8, 512, 2), (6, 12): (4, 512, 4), (6, 13): (1, 512, 16),
                (6, 14): (4, 512, 4)}


def kernel_name(b, variant):
    if b == 7:
        return "k_numeric_mpass + k_finish_mpass (multi-pass sliced tables)"
    if (b, variant) in SPLIT_SHAPES:
        nw, sw, p = SPLIT_SHAPES[(b, variant)]
        return ("k_numeric_part<%d waves x %d slots, %d parts per column> (bin %d accumulation; "
                "k_finish_part sorts and prunes)" % (nw, sw, p, b))
    if b >= 3 and variant == 0:
        return "k_numeric_hsplit<%d waves, 512 slots each> (bin %d)" % (1 << (b - 2), b)
    return "k_numeric_lds<%d slots> (bin %d, launch variant %d)" % (128 << b, b, variant)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, target_s=12.0, seed=7, single_s=6.0):
    """The CPU oracle (expand + prune + inflate) on a random sample of columns
    of the same column-stochastic A the GPU iterated (downloaded from the
    device), on all threads and on one thread.  Returns the baseline record
    and the sample (columns, unpruned product, prune info, result) for the
    parity check of the GPU output."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    n = A.ncols

    def run(frac):
        cols = np.sort(rng.choice(n, size=max(1, int(frac * n)), replace=False))
        Bs = A.restrict_columns(cols)
        t = time.perf_counter()
        C, flops, nnz = oracle.expand(A, Bs)
        P, info = oracle.prune(C)
        I = oracle.inflate(P, 2.0)
        return time.perf_counter() - t, int(flops.sum()), int(nnz.sum()), cols, C, info, I

    threads = oracle.num_threads()
    dt, fl, nz, cols, _, _, _ = run(0.002)
    frac = min(1.0, 0.002 * target_s / max(dt, 1e-3))
    dt, fl, nz, cols, C, info, I = run(frac)
    rec = {"value": round(fl / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "%d of %d columns (uniform, seed %d) of the GPU's normalised input: "
                     "expand+prune+inflate, %.1f s on %d threads, %.3g multiply-adds, %.3g product nnz/s"
                     % (len(cols), n, seed, dt, threads, fl, nz / dt)}
    # single thread, on a smaller sample of the same kind
    oracle.set_num_threads(1)
    try:
        dt1, fl1, _, cols1, _, _, _ = run(min(1.0, frac * single_s / max(dt * threads, 1e-3)))
    finally:
        oracle.set_num_threads(threads)
    rec["single_thread"] = {"value": round(fl1 / dt1 / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
                            "sample": "%d columns, %.1f s" % (len(cols1), dt1)}
    return rec, (cols, C, info, I)


def gpu_parity(G, sample, theta=1e-4, pct=0.9, rtol=1e-12):
    """Compares the GPU's fused iteration on the sampled columns with the
    oracle's expand + prune + inflate of the same columns: row patterns must
    be identical and values within rtol, except where a column's kept set
    differs only by entries within 1e-12 (relative) of its threshold, or its
    recovery test is within 1e-12 of equality (near-ties, accepted either
    way)."""
    import numpy as np
    import torch
    cols, C, info, I = sample
    ct = torch.from_numpy(cols.astype(np.int64)).to(G.colptr.device)
    s = G.colptr[ct]
    cnt = G.colptr[ct + 1] - s
    total = int(cnt.sum())
    start = torch.cumsum(cnt, 0) - cnt
    idx = torch.repeat_interleave(s - start, cnt) + torch.arange(total, device=s.device)
    grow = G.rowidx[idx].cpu().numpy()
    gval = G.val[idx].cpu().numpy()
    gcnt = cnt.cpu().numpy()
    gcp = np.zeros(len(cols) + 1, np.int64)
    gcp[1:] = np.cumsum(gcnt)
    ocnt = np.diff(I.colptr)
    same_len = gcnt == ocnt
    # columns of equal length: compare rows in bulk
    col_of = np.repeat(np.arange(len(cols)), ocnt)
    eq_len_entry = same_len[col_of]
    gpos = (gcp[:-1] - I.colptr[:-1])[col_of] + np.arange(I.nnz)
    row_ok = np.ones(I.nnz, bool)
    row_ok[eq_len_entry] = grow[gpos[eq_len_entry]] == I.rowidx[eq_len_entry]
    bad_col = ~same_len
    np.logical_or.at(bad_col, col_of, ~row_ok)
    good_entry = ~bad_col[col_of]
    rel = np.abs(gval[gpos[good_entry]] - I.val[good_entry]) / I.val[good_entry]
    max_rel = float(rel.max(initial=0.0))
    bad_val = int((rel > rtol).sum())
    near = unexplained = 0
    for q in np.nonzero(bad_col)[0]:
        mB, mP, t = info["mass"][q], info["mass_above"][q], info["threshold"][q]
        gq = grow[gcp[q]:gcp[q + 1]]
        gr = set(gq.tolist())
        orr = set(I.rowidx[I.colptr[q]:I.colptr[q + 1]].tolist())
        # a near-tie changes the kept set; rows out of order or repeated never pass
        ok = gr != orr and bool(np.all(np.diff(gq) > 0))
        if ok and not abs(mP - pct * mB) <= 1e-12 * mB:
            r0, v0 = C.column(q)
            vals = dict(zip(r0.tolist(), v0.tolist()))
            ok = all(r in vals and (abs(vals[r] - t) <= 1e-12 * t or abs(vals[r] - theta) <= 1e-12 * theta)
                     for r in gr ^ orr)
        near += ok
        unexplained += not ok
    return {"columns": int(len(cols)), "entries": int(I.nnz), "mismatches": unexplained + bad_val,
            "near_tie_columns": near, "max_rel_diff": max_rel, "rtol": rtol,
            "rule": "row patterns identical, values within rtol; kept sets may differ only by "
                    "entries within 1e-12 of the column threshold (near-ties)"}


def _line(metric, value, unit, ms, higher, workload, extra, steps=1, warmup=0, dtype="f64"):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": round(ms, 3), "higher_is_better": higher, "scaling": "strong", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic", "config": {"workload": workload}}
    d.update(extra)
    return d


def bench_merge(args, sample_cols=4096, seed=11):
    """One process's share of a 2D Sparse SUMMA product (Section 2 "Overview
    of Sparse SUMMA", Section 4 and Alg. 2) at its real block shape: the
    planted graph on 10,000,000 vertices (~480 nnz/column, seed 1002) on an
    8 x 8 process grid, position (0, 1): 8 stage products A[0,k] * A[k,1] of
    1.25M x 1.25M blocks (~60 nnz/column each), the partials merged by the
    binary schedule (Alg. 2) or all at once, with the merges on the same stream
    as the products or on a second stream overlapped with them."""
    import numpy as np
    import torch
    import oracle
    from mclgen.planted import stripe_blocks
    from paper_2002_10083_amd import drivers, mcl, tuning
    t0 = time.time()
    R, Cb = stripe_blocks(N=args.merge_n, grid=8, row_stripe=0, col_stripe=1, workers=16)
    log("generated 16 blocks of %d x %d in %.1f s (nnz %s / %s)" % (R[0].nrows, R[0].ncols, time.time() - t0,
                                                                   [x.nnz for x in R], [x.nnz for x in Cb]))
    dR = [mcl.DeviceCSC.from_host(x) for x in R]
    dC = [mcl.DeviceCSC.from_host(x) for x in Cb]
    torch.cuda.synchronize()
    policy, scale, keys = tuning.load_policy("iterate")
    params = mcl.default_params(bin_policy=policy, est_scale=scale, cohen_keys=keys)

    def operands(i):
        return dR[i], dC[i]

    res, keep = {}, {}
    # the first two runs warm up (kernels, and torch's cache grows to the
    # larger peak once: fresh device memory is slow to map on first use, so
    # the cache is kept between runs)
    plan = [("flat", False), ("binary", False), ("binary", False), ("flat", False), ("binary", True),
            ("flat", True)]
    for n, (sched, ov) in enumerate(plan):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        run = drivers.summa_stages_overlapped if ov else drivers.summa_stages
        ms0 = torch.cuda.memory_stats()
        C, info = run(operands, 8, sched, params)
        ms1 = torch.cuda.memory_stats()
        info["peak_device_bytes"] = int(torch.cuda.max_memory_allocated() - base)
        info["alloc_retries"] = int(ms1.get("num_alloc_retries", 0) - ms0.get("num_alloc_retries", 0))
        info["device_allocs"] = int(ms1.get("num_device_alloc", 0) - ms0.get("num_device_alloc", 0))
        key = sched + ("_overlap" if ov else "")
        res[key] = info
        log("%s: expand %.1f ms, merge %.1f ms, wall %.1f ms, peak %.2f GB, nnz %d, alloc retries %d, "
            "device allocs %d" % (key, info["t_expand_ms"], info["t_merge_ms"], info["wall_ms"],
                                  info["peak_device_bytes"] / 1e9, info["nnz"], info["alloc_retries"],
                                  info["device_allocs"]))
        for c in info["merge_calls"]:
            log("   merge of %d lists: in %d out %d, %.1f ms, bins ms %s cols %s" %
                (c["lists"], c["in_nnz"], c["out_nnz"], c["ms"], [round(x, 1) for x in c["bin_ms"]],
                 c["bin_cols"]))
        if n > 1 and not ov:
            # sampled output columns for the parity check against the oracle
            rng = np.random.default_rng(seed)
            cols = np.sort(rng.choice(C.ncols, size=min(sample_cols, C.ncols), replace=False))
            keep[sched] = _download_columns(C, cols)
        del C
    # parity on sampled columns: the oracle's stage products of those columns,
    # merged by the oracle's heap merge with the same schedule
    t1 = time.time()
    cols = keep["binary"][0]
    parts = [oracle.expand(R[k], Cb[k].restrict_columns(cols))[0] for k in range(8)]
    ref_b, _ = oracle.binary_merge(parts)
    ref_f = oracle.merge(parts)
    par = {}
    for sched, ref in (("binary", ref_b), ("flat", ref_f)):
        _, cp, row, val = keep[sched]
        same = np.array_equal(cp, ref.colptr) and np.array_equal(row, ref.rowidx) and np.array_equal(val, ref.val)
        par[sched] = {"columns": int(len(cols)), "entries": int(ref.nnz), "bit_identical": bool(same)}
    log("merge parity took %.1f s: %s" % (time.time() - t1, par))
    b, bo, f = res["binary"], res["binary_overlap"], res["flat"]
    merged_in = sum(c["in_nnz"] for c in b["merge_calls"])
    mb = sum(c["bytes"] for c in b["merge_calls"])
    mms = sum(c["ms"] for c in b["merge_calls"])
    roof = {"bound": "hbm", "achieved": round(mb / (mms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(mb / (mms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "merge calls of the binary schedule (sequential run)", "ms": round(mms, 3),
            "algorithmic_bytes": int(mb)}
    pick = ("t_expand_ms", "t_merge_ms", "wall_ms", "peak_list_bytes", "peak_device_bytes", "merges", "nnz")
    out = {k: {q: res[k][q] for q in pick} for k in res}
    for k in ("binary_overlap", "flat_overlap"):
        out[k]["overlap_frac"] = round(res[k]["overlap_frac"], 4)
    return _line("SUMMA stage products + merge at the real block shape: partial-product nnz merged per s "
                 "(binary schedule, overlapped)",
                 round(merged_in / (bo["wall_ms"] * 1e-3), 1), "nnz/s", bo["wall_ms"], True,
                 "one process's share of a 10M-vertex planted graph on an 8x8 grid (position (0,1), seed 1002): "
                 "8 products of 1.25M x 1.25M blocks, partials merged by Alg. 2 vs one 8-way merge, "
                 "on one stream or overlapped on two",
                 {"runs": out, "partial_nnz": b["partial_nnz"],
                  "expand_flops_note": "see stage sizes", "merge_roofline": roof,
                  "merge_share_binary": round(b["t_merge_ms"] / b["wall_ms"], 4),
                  "time_binary_over_flat": round(b["wall_ms"] / f["wall_ms"], 4),
                  "peak_list_bytes_binary_over_flat": round(b["peak_list_bytes"] / f["peak_list_bytes"], 4),
                  "wall_overlapped_over_sequential": round(bo["wall_ms"] / b["wall_ms"], 4),
                  "parity": par})


def _download_columns(C, cols):
    """Host copies of the given columns of a device CSC: (cols, colptr, rows, values)."""
    import numpy as np
    import torch
    ct = torch.from_numpy(cols.astype(np.int64)).to(C.colptr.device)
    s = C.colptr[ct]
    cnt = C.colptr[ct + 1] - s
    total = int(cnt.sum())
    start = torch.cumsum(cnt, 0) - cnt
    idx = torch.repeat_interleave(s - start, cnt) + torch.arange(total, device=s.device)
    cp = np.zeros(len(cols) + 1, np.int64)
    cp[1:] = np.cumsum(cnt.cpu().numpy())
    return cols, cp, C.rowidx[idx].cpu().numpy(), C.val[idx].cpu().numpy()


def bench_batched(args, seed=5):
    """MCL to convergence over the 20,000-component block-diagonal graph:
    all components per call (converged ones frozen) vs the plain loop, one
    component at a time, over every component (or a stratified sample with
    --loop-sample: every component above 2,000 vertices plus a uniform sample
    of the rest, scaled by its inverse sampling rate)."""
    import numpy as np
    import torch
    from mclgen import config3_graph
    from paper_2002_10083_amd import drivers, mcl, tuning
    t0 = time.time()
    U = config3_graph()
    log("generated %d components, n=%d nnz=%d in %.1f s" % (len(U.comp_ptr) - 1, U.ncols, U.nnz,
                                                           time.time() - t0))
    A = mcl.DeviceCSC.from_host(U)
    mcl.normalize_(A)
    comp = torch.from_numpy(U.comp_ptr).cuda()
    key = "batched" if tuning.has_policy("batched") else "iterate"
    policy, scale, keys = tuning.load_policy(key)
    params = mcl.default_params(bin_policy=policy, est_scale=scale, cohen_keys=keys)
    An = A.to_host()
    torch.cuda.synchronize()
    t = time.perf_counter()
    Af, iters, info = drivers.batched_mcl(A, comp, params)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t
    log("batched: %.2f s, %d calls, not converged %d" % (t_batched, info["calls"], info["not_converged"]))
    # the other accumulation schedule of the same run: one persistent launch
    # for all LDS bins per iteration when the tuned policy uses per-bin
    # launches (and the reverse), same results
    alt_policy = policy ^ tuning.PERSIST
    torch.cuda.synchronize()
    t = time.perf_counter()
    Aalt, iters_alt, info_alt = drivers.batched_mcl(A, comp, mcl.default_params(bin_policy=alt_policy,
                                                                               est_scale=scale, cohen_keys=keys))
    torch.cuda.synchronize()
    t_alt = time.perf_counter() - t
    alt_same = (np.array_equal(iters_alt, iters) and torch.equal(Aalt.colptr, Af.colptr)
                and torch.equal(Aalt.rowidx, Af.rowidx) and torch.equal(Aalt.val, Af.val))
    del Aalt
    log("batched with persistent accumulation %s: %.2f s, identical %s"
        % ("on" if alt_policy & tuning.PERSIST else "off", t_alt, alt_same))
    ncomp = len(U.comp_ptr) - 1
    sizes = np.diff(U.comp_ptr)
    if args.loop_sample > 0:
        rng = np.random.default_rng(seed)
        big = np.nonzero(sizes > 2000)[0]
        small = np.nonzero(sizes <= 2000)[0]
        pick_small = rng.choice(small, size=min(args.loop_sample, len(small)), replace=False)
        pick = np.sort(np.concatenate([big, pick_small]))
        weight = np.where(sizes[pick] > 2000, 1.0, len(small) / max(1, len(pick_small)))
    else:
        pick = np.arange(ncomp)
        weight = np.ones(ncomp)
    t_loop = 0.0
    same = 0
    tl0 = time.time()
    for n, c in enumerate(pick):
        c0, c1 = int(U.comp_ptr[c]), int(U.comp_ptr[c + 1])
        blk = mcl.DeviceCSC.from_host(drivers.component_block(An, c0, c1))
        torch.cuda.synchronize()
        t = time.perf_counter()
        Bf, it, _ = drivers.component_mcl(blk, params)
        torch.cuda.synchronize()
        t_loop += (time.perf_counter() - t) * weight[n]
        same += int(bool(it == iters[c]) and drivers.same_block(Af, c0, c1, Bf))
        if (n + 1) % 2000 == 0:
            log("loop: %d of %d components, %.1f s" % (n + 1, len(pick), time.time() - tl0))
    return _line("MCL to convergence over 20,000 components: batched speedup over the per-component loop",
                 round(t_loop / t_batched, 3), "x", t_batched * 1e3, True,
                 "block-diagonal planted graph, 20,000 components of 8..30,000 vertices (seed 1003)",
                 {"n": U.ncols, "nnz": U.nnz, "components": ncomp, "batched_s": round(t_batched, 3),
                  "batched_calls": info["calls"], "iterations_max": int(iters.max()),
                  "iterations_mean": round(float(iters.mean()), 2), "not_converged": info["not_converged"],
                  "policy_key": key, "bin_policy": hex(policy),
                  "persistent_accumulation": bool(policy & tuning.PERSIST),
                  "other_schedule": {"persistent_accumulation": bool(alt_policy & tuning.PERSIST),
                                     "batched_s": round(t_alt, 3), "identical": bool(alt_same)},
                  "loop_components_timed": int(len(pick)),
                  "loop_s": round(t_loop, 3),
                  "loop_mode": "all components" if args.loop_sample <= 0 else
                               "components above 2,000 vertices + %d sampled below, weighted" % args.loop_sample,
                  "bit_identical_components": int(same),
                  "per_call_ms": [round(s_["ms"], 2) for s_ in info["steps"]]})


def bench_mlp(args, cfg1_seeds=tuple(range(2001, 2009)), cfg3_seeds=(2101, 2102), heldout_seed=2009,
              scales=(0.7, 0.85, 1.0, 1.2, 1.45, 1.75), reps=3):
    """Learned table sizing.  Training rows are logged from the method's own
    runs on graphs of the benchmark's shapes with other seeds (1M-vertex
    planted graphs, 4 iterations each, and 20,000-component graphs, 3
    iterations each); the MLP is trained with the library's kernels; its
    sizing margin is the 0.75-quantile of its log residual on a held-out
    1M-vertex graph (Cohen's margin is the tuned one).  Then the fused
    iteration on the benchmark graph (seed 1001) runs with each estimator the
    same number of times, plus the same sweep of margins for both."""
    import numpy as np
    import torch
    from mclgen import config1_graph, config3_graph
    from paper_2002_10083_amd import learned, mcl, tuning
    policy, scale, keys = tuning.load_policy("iterate")
    base = dict(bin_policy=policy, cohen_keys=keys)
    cohen_kw = dict(estimator=mcl.EST_COHEN)
    Xs, ys = [], []
    t = time.time()
    shapes = [("1M-vertex planted", sd, 4) for sd in cfg1_seeds] + [("20,000 components", sd, 3) for sd in cfg3_seeds]
    for kind, sd, its in shapes:
        W = config1_graph(seed=sd) if kind.startswith("1M") else config3_graph(seed=sd)
        At = mcl.DeviceCSC.from_host(W)
        del W
        mcl.normalize_(At)
        X, y = learned.collect(At, iterations=its, params=mcl.default_params(**base, est_scale=scale))
        Xs.append(X)
        ys.append(y)
        del At
        log("collected %s seed %d: %d rows (%.1f s)" % (kind, sd, X.shape[0], time.time() - t))
    X, y = torch.cat(Xs), torch.cat(ys)
    del Xs, ys
    t_collect = time.time() - t
    torch.cuda.synchronize()
    t = time.perf_counter()
    state, packed, losses = learned.train(X, y, epochs=6, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    rows_per_s = X.shape[0] * 6 / t_train
    n_rows = int(X.shape[0])
    del X, y
    mlp_kw = dict(estimator=mcl.EST_MLP, mlp_weights=packed)
    # sizing margins from held-out residuals (iteration 0, the benchmark's)
    H = mcl.DeviceCSC.from_host(config1_graph(seed=heldout_seed))
    mcl.normalize_(H)
    hp = mcl.default_params(**base, est_scale=scale)
    q_mlp = learned.residual_quantiles(H, dict(mlp_kw), iterations=1, params=hp)
    q_cohen = learned.residual_quantiles(H, dict(cohen_kw, cohen_keys=keys), iterations=1, params=hp)
    del H
    mlp_scale = learned.scale_for_quantile(q_mlp, 0.75)
    log("held-out residual quantiles: mlp %s cohen %s -> mlp est_scale %.3f" % (q_mlp, q_cohen, mlp_scale))
    W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)
    pick = ("t_total_ms", "t_symbolic_ms", "t_estimate_ms", "t_numeric_ms", "t_fallback_ms", "n_overflow",
            "n_global")

    def run(kw, sc, n):
        best, outs = None, None
        for _ in range(n):
            G, ch, st = mcl.iterate(A, mcl.default_params(**dict(base, **kw), est_scale=sc))
            if best is None or st["t_total_ms"] < best["t_total_ms"]:
                best = st
            outs = G
        return outs, dict({k: best[k] for k in pick}, est_scale=round(sc, 4))

    Gc, sc_ = run(cohen_kw, scale, reps)
    Gm, sm = run(mlp_kw, mlp_scale, reps)
    same = torch.equal(Gc.rowidx, Gm.rowidx) and torch.equal(Gc.val, Gm.val) and torch.equal(Gc.colptr, Gm.colptr)
    del Gc, Gm
    sweep = {"cohen": [], "mlp": []}
    for name, kw in (("cohen", cohen_kw), ("mlp", mlp_kw)):
        for sc in scales:
            _, st = run(kw, sc, 2)
            sweep[name].append(st)
    best_c = min(sweep["cohen"], key=lambda d: d["t_total_ms"])
    best_m = min(sweep["mlp"], key=lambda d: d["t_total_ms"])
    acc = learned.evaluate(packed, A)
    return _line("fused MCL iteration at n=1M: speedup of learned (MLP) table sizing over Cohen",
                 round(sc_["t_total_ms"] / sm["t_total_ms"], 4), "x", sm["t_total_ms"], True,
                 "one fused MCL iteration on the 1M-vertex planted graph (seed 1001); MLP trained on %d "
                 "rows from 1M-vertex planted graphs (seeds %d-%d, 4 iterations) and 20,000-component "
                 "graphs (seeds %s, 3 iterations); margin from held-out seed %d"
                 % (n_rows, cfg1_seeds[0], cfg1_seeds[-1], list(cfg3_seeds), heldout_seed),
                 {"cohen": sc_, "mlp": sm, "bit_identical": bool(same), "runs_each": reps,
                  "margin_rule": "est_scale = exp(Q0.75 of held-out log residual) / 1.3",
                  "heldout_residual_quantiles": {"mlp": q_mlp, "cohen": q_cohen},
                  "sweep": sweep,
                  "best_of_sweep_speedup": round(best_c["t_total_ms"] / best_m["t_total_ms"], 4),
                  "train_rows": n_rows, "train_rows_per_s": round(rows_per_s, 1),
                  "collect_s": round(t_collect, 1), "train_s": round(t_train, 2),
                  "loss_first_last": [round(losses[0], 4), round(losses[-1], 4)],
                  "log_error": acc}, dtype="bf16/f32 MLP, f64 expansion")


def bench_dispatch(args, sizes=(100, 200, 300, 500, 700, 1000, 1500, 2000, 4000, 16000, 64000), reps=5):
    """The CPU/GPU dispatch by flops (host matrices in and out): the CPU hash
    SpGEMM on every host thread against the GPU expansion including both
    copies, on planted graphs of growing size.  The flops where the GPU leg
    becomes faster is the dispatch threshold.  Also the host SpGEMM's rate on
    the 1M-vertex benchmark graph, next to the oracle's."""
    import numpy as np
    import torch
    from mclgen import config1_graph
    from paper_2002_10083_amd import mcl
    rows = []
    for i, n in enumerate(sizes):
        A = mcl.DeviceCSC.from_host(config1_graph(seed=4000 + i, n=n, n_clusters=max(1, n // 20)))
        mcl.normalize_(A)
        H = A.to_host()
        t = {}
        outs = {}
        for leg, cut in (("cpu", 1 << 62), ("gpu", 1)):
            best = None
            for _ in range(reps):
                C, st, where = mcl.expand_dispatch(H, H, gpu_min_flops=cut)
                assert where == leg
                best = st["t_total_ms"] if best is None else min(best, st["t_total_ms"])
            t[leg] = best
            outs[leg] = C
            fl = st["flops"]
        same = (np.array_equal(outs["cpu"].rowidx, outs["gpu"].rowidx)
                and np.array_equal(outs["cpu"].val.view(np.uint64), outs["gpu"].val.view(np.uint64)))
        rows.append({"n": n, "flops": int(fl), "cpu_ms": round(t["cpu"], 3), "gpu_ms": round(t["gpu"], 3),
                     "bit_identical": bool(same)})
        log("dispatch n=%d flops=%.3g cpu %.2f ms gpu %.2f ms same=%s" % (n, fl, t["cpu"], t["gpu"], same))
    # crossover: between the largest product the CPU leg still wins and the
    # next larger one (geometric mean of their flops)
    by = sorted(rows, key=lambda r: r["flops"])
    last_cpu = max((i for i, r in enumerate(by) if r["cpu_ms"] < r["gpu_ms"]), default=None)
    if last_cpu is None:
        cross = None  # the GPU leg wins at every size measured
    elif last_cpu + 1 < len(by):
        cross = float(np.sqrt(by[last_cpu]["flops"] * by[last_cpu + 1]["flops"]))
    else:
        cross = float(by[-1]["flops"])
    W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)
    H = A.to_host()
    del W
    t = time.perf_counter()
    C, st = mcl.expand_host(H, H)
    host_s = time.perf_counter() - t
    host_rate = st["flops"] / (st["t_total_ms"] * 1e6)
    G, gst = mcl.expand(A, A)
    same = (np.array_equal(C.colptr, G.colptr.cpu().numpy()) and np.array_equal(C.rowidx, G.rowidx.cpu().numpy())
            and np.array_equal(C.val.view(np.uint64), G.val.cpu().numpy().view(np.uint64)))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return _line("host hash SpGEMM GFLOP/s at n=1M and the CPU/GPU dispatch crossover", round(host_rate, 3),
                 "GFLOP/s", st["t_total_ms"], True,
                 "expansion A*A of the 1M-vertex planted graph (seed 1001) on the host's threads; dispatch "
                 "sweep on planted graphs of %d..%d vertices" % (sizes[0], sizes[-1]),
                 {"host_threads": threads, "cpu_model": cpu_model(), "host_wall_s": round(host_s, 2),

                  "gpu_expand_ms": round(gst["t_total_ms"], 3),
                  "gpu_GFLOPs": round(gst["flops"] / (gst["t_total_ms"] * 1e6), 2),
                  "bit_identical_vs_gpu": bool(same), "sweep": rows,
                  "crossover_flops": None if cross is None else round(cross)})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--estimator", default="cohen", choices=["cohen", "bound"])
    ap.add_argument("--policy", type=lambda x: int(x, 0), default=None,
                    help="bin launch policy (default: tuned table if present)")
    ap.add_argument("--est-scale", type=float, default=None,
                    help="table sizing margin (default: the tuned one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--loop-sample", type=int, default=0,
                    help="batched workload: 0 times the plain loop over every component; k > 0 times every "
                         "component above 2,000 vertices and k sampled below")
    ap.add_argument("--merge-n", type=int, default=10_000_000,
                    help="merge workload: vertices of the whole graph (8 x 8 grid)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--workload", default="iterate", choices=["iterate", "merge", "batched", "mlp", "dispatch"],
                    help="iterate: one fused iteration at n=1M (default); merge: 8 SUMMA-stage "
                         "partials merged by Alg. 2 vs one flat merge; batched: MCL to convergence "
                         "over 20,000 components, batched vs per component; mlp: learned vs Cohen "
                         "table sizing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload != "iterate":
        import torch
        torch.cuda.set_device(0)
        out = {"merge": bench_merge, "batched": bench_batched, "mlp": bench_mlp,
               "dispatch": bench_dispatch}[args.workload](args)
        print(json.dumps(out), flush=True)
        return

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
    if args.est_scale is not None:
        scale = args.est_scale
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
    G = None
    for i in range(args.steps):
        del G
        G, change, st = mcl.iterate(A, params)
        sts.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ms_step = dt / args.steps * 1e3
    flops = sts[0]["flops"]
    nnz_prod = sts[0]["nnz_product"]
    kept = sts[0]["nnz_kept"]
    gflops = flops * args.steps / dt / 1e9

    # dominant kernel: the bin with the largest mean time over the timed steps;
    # for a split bin, its accumulation kernel (the finishing kernel is reported beside it)
    nb = 8
    mean_ms = [float(np.mean([s["bin_ms"][b] for s in sts])) for b in range(nb)]
    part_ms = [float(np.mean([s["bin_part_ms"][b] for s in sts])) for b in range(nb)]
    dom = int(np.argmax(mean_ms))
    variant = (policy >> (4 * dom)) & 15 if dom < 7 else 0
    name = kernel_name(dom, variant)
    kernel_key = "bin%d-v%d-keys%d" % (dom, variant, keys)
    if part_ms[dom] > 0:
        byt = part_bytes(sts[0], dom)
        kms = part_ms[dom]
    else:
        byt = bin_bytes(sts[0], dom)
        kms = mean_ms[dom]
    achieved = byt / (kms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel_key),
            "kernel": name, "kernel_key": kernel_key,
            "kernel_ms": round(kms, 3), "algorithmic_bytes": int(byt)}
    if part_ms[dom] > 0:
        bb = bin_bytes(sts[0], dom)
        roof["bin_with_finish"] = {"ms": round(mean_ms[dom], 3), "finish_ms": round(mean_ms[dom] - kms, 3),
                                   "algorithmic_bytes": int(bb),
                                   "frac": round(bb / (mean_ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
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
    out["bins"] = [{"bin": b, "cols": sts[0]["bin_cols"][b], "flops": sts[0]["bin_flops"][b],
                    "ms": round(mean_ms[b], 3), "accum_ms": round(part_ms[b], 3),
                    "algorithmic_GBps": round(bin_bytes(sts[0], b) / max(mean_ms[b], 1e-9) / 1e6, 1)}
                   for b in range(nb)]
    log("bins ms:", [round(x, 2) for x in mean_ms])
    log("split accumulation ms:", [round(x, 2) for x in part_ms])
    if not args.no_cpu_baseline:
        t1 = time.time()
        out["cpu_baseline"], sample = cpu_baseline(A.to_host())
        log("cpu baseline took %.1f s" % (time.time() - t1))
        t1 = time.time()
        out["parity"] = gpu_parity(G, sample)
        log("parity check took %.1f s: %s" % (time.time() - t1, out["parity"]))
    else:
        out["cpu_baseline"] = None
        out["parity"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
