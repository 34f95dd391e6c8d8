"""Host-side drivers over the C-ABI calls (argument handling and loop control
only; every arithmetic step runs in the library's kernels).

* ``summa_merge`` / ``summa_stages`` / ``summa_stages_overlapped``: the
  inner dimension of C = A*A (or given stage operand pairs) is cut into ``nstages``
  contiguous ranges K_1..K_s, stage i contributes the partial product
  A[:, K_i] * A[K_i, :] (one SUMMA stage of one process, Section 4), and the
  partials are merged either with the binary schedule of Alg. 2 (after stage
  i, the top 1 + v2(i) lists of the stack are merged, v2 = number of factors
  of two) or all at once after the last stage.  Equal rows are summed in
  stage order.
* ``batched_mcl`` / ``component_mcl``: MCL to convergence over a
  block-diagonal matrix of many components, either all components in each
  call with a per-component active mask, or one component at a time.
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np
import torch

from . import mcl


def csc_bytes(M: "mcl.DeviceCSC") -> int:
    return 8 * (M.ncols + 1) + 12 * M.nnz


def stage_ranges(n: int, nstages: int):
    """Contiguous ranges of the inner dimension, one per stage (sizes differ by <= 1)."""
    cuts = [(n * i) // nstages for i in range(nstages + 1)]
    return [(cuts[i], cuts[i + 1]) for i in range(nstages)]


def column_block(A: "mcl.DeviceCSC", k0: int, k1: int) -> "mcl.DeviceCSC":
    """A[:, k0:k1] (views of A's row and value arrays)."""
    cp = A.colptr[k0:k1 + 1]
    p0, p1 = int(cp[0]), int(cp[-1])
    return mcl.DeviceCSC(A.nrows, k1 - k0, (cp - p0).contiguous(), A.rowidx[p0:p1], A.val[p0:p1])


def row_block(A: "mcl.DeviceCSC", k0: int, k1: int) -> "mcl.DeviceCSC":
    """A[k0:k1, :] with rows renumbered from 0 (rows stay ascending)."""
    keep = (A.rowidx >= k0) & (A.rowidx < k1)
    counts = torch.diff(A.colptr)
    col = torch.repeat_interleave(torch.arange(A.ncols, device=A.colptr.device), counts)
    per_col = torch.bincount(col[keep], minlength=A.ncols)
    cp = torch.zeros(A.ncols + 1, dtype=torch.int64, device=A.colptr.device)
    cp[1:] = torch.cumsum(per_col, 0)
    return mcl.DeviceCSC(k1 - k0, A.ncols, cp, (A.rowidx[keep] - k0).to(torch.int32).contiguous(),
                         A.val[keep].contiguous())


def binary_schedule(nstages: int) -> List[int]:
    """Lists merged after each stage by Alg. 2 (0 = none)."""
    out = []
    for i in range(1, nstages + 1):
        v = (i & -i).bit_length() - 1
        out.append(v + 1 if v > 0 else 0)
    return out


def summa_merge(A: "mcl.DeviceCSC", nstages: int = 8, schedule: str = "binary", params=None,
                overlap: bool = False):
    """C = sum over stages of A[:, K_i] A[K_i, :], merged per `schedule`
    ("binary" = Alg. 2, "flat" = one merge of all partials at the end).
    Returns (C, info) with expansion and merge times (ms), the peak bytes held
    by partial and merged lists, and the per-stage list sizes."""
    ranges = stage_ranges(A.ncols, nstages)

    def operands(i):
        k0, k1 = ranges[i]
        return column_block(A, k0, k1), row_block(A, k0, k1)

    if overlap:
        return summa_stages_overlapped(operands, nstages, schedule, params)
    return summa_stages(operands, nstages, schedule, params)


def summa_stages(operands, nstages: int, schedule: str = "binary", params=None):
    """One process's Sparse SUMMA stages on one stream: stage i multiplies the
    pair operands(i) = (A_i, B_i) (same output shape for every stage) and the
    partial products are merged per `schedule` (see summa_merge).  Returns
    (C, info) as summa_merge."""
    if schedule not in ("binary", "flat"):
        raise ValueError(schedule)
    stack: List[mcl.DeviceCSC] = []
    live = peak = 0
    t_exp = t_mrg = 0.0
    sizes = []
    merges = []

    calls = []

    def merge(lists):
        nonlocal live, peak, t_mrg
        torch.cuda.synchronize()
        t = time.perf_counter()
        M, st = mcl.merge_partials(lists)
        torch.cuda.synchronize()
        t_mrg += (time.perf_counter() - t) * 1e3
        peak = max(peak, live + csc_bytes(M))
        live += csc_bytes(M) - sum(csc_bytes(x) for x in lists)
        merges.append(len(lists))
        calls.append(merge_call_info(lists, M, st))
        return M

    plan = binary_schedule(nstages)
    t_wall = time.perf_counter()
    for i in range(1, nstages + 1):
        Ak, Bk = operands(i - 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        P, _ = mcl.expand(Ak, Bk, params)
        torch.cuda.synchronize()
        t_exp += (time.perf_counter() - t) * 1e3
        del Ak, Bk
        stack.append(P)
        sizes.append(P.nnz)
        live += csc_bytes(P)
        peak = max(peak, live)
        if schedule == "binary" and plan[i - 1] > 0:
            take = stack[-plan[i - 1]:]
            del stack[-plan[i - 1]:]
            stack.append(merge(take))
            del take
    if len(stack) > 1:
        M = merge(stack)
        stack = [M]
    C = stack[0]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) * 1e3
    return C, dict(t_expand_ms=t_exp, t_merge_ms=t_mrg, peak_list_bytes=peak, partial_nnz=sizes,
                   merges=merges, nnz=C.nnz, wall_ms=wall, overlap=False, merge_calls=calls)


def merge_call_info(lists, M, st):
    """One merge call: list sizes, output size, the library's event time and
    its algorithmic bytes (every input entry read once, 12 B, plus its colptr
    pair, 16 B per column and list; every output entry written once, 12 B,
    plus 8 B per column)."""
    nin = sum(x.nnz for x in lists)
    byt = 12 * nin + 16 * M.ncols * len(lists) + 12 * M.nnz + 8 * (M.ncols + 1)
    return dict(lists=len(lists), in_nnz=nin, out_nnz=M.nnz, ms=st["t_merge_ms"], bytes=byt,
                bin_ms=st["bin_ms"], bin_cols=st["bin_cols"])


def summa_stages_overlapped(operands, nstages: int, schedule: str = "binary", params=None):
    """summa_stages with the merges on a second stream, run by a host thread
    of their own: the merge Alg. 2 schedules after stage i runs while stage
    i+1 is multiplied on the caller's stream (the paper's pipelining of the
    merge against the local multiplications, Section 3 and Section 4).  A
    merge waits for the event recorded after the stage that produced its last
    list; merges run in schedule order, so the lists an earlier merge produced
    are complete.  Returns (C, info) as summa_merge, plus the busy time of
    each stream, the wall time and the fraction of the merge time hidden
    behind the products (overlap_frac = (t_expand + t_merge - wall) /
    t_merge)."""
    import threading
    from concurrent.futures import Future, ThreadPoolExecutor

    if schedule not in ("binary", "flat"):
        raise ValueError(schedule)
    dev = torch.cuda.current_device()
    s_merge = torch.cuda.Stream(device=dev)      # default priority
    lock = threading.Lock()
    acct = dict(t_mrg=0.0, live=0, peak=0)
    calls = []
    merges: List[int] = []
    sizes: List[int] = []

    def add_live(delta):
        with lock:
            acct["live"] += delta
            acct["peak"] = max(acct["peak"], acct["live"])

    def run_merge(inputs, ready):
        torch.cuda.set_device(dev)
        lists = [x.result() if isinstance(x, Future) else x for x in inputs]
        with torch.cuda.stream(s_merge):
            s_merge.wait_event(ready)
            t = time.perf_counter()
            M, st = mcl.merge_partials(lists)
            s_merge.synchronize()
            dt = (time.perf_counter() - t) * 1e3
        with lock:
            acct["t_mrg"] += dt
            calls.append(merge_call_info(lists, M, st))
        add_live(csc_bytes(M))
        add_live(-sum(csc_bytes(x) for x in lists))
        del lists, inputs
        return M

    plan = binary_schedule(nstages)
    stack = []
    t_exp = 0.0
    s_main = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    with ThreadPoolExecutor(max_workers=1) as ex:
        for i in range(1, nstages + 1):
            Ak, Bk = operands(i - 1)
            t = time.perf_counter()
            P, _ = mcl.expand(Ak, Bk, params)
            s_main.synchronize()
            t_exp += (time.perf_counter() - t) * 1e3
            del Ak, Bk
            ev = torch.cuda.Event()
            ev.record(s_main)
            sizes.append(P.nnz)
            add_live(csc_bytes(P))
            stack.append(P)
            del P
            if schedule == "binary" and plan[i - 1] > 0:
                take = stack[-plan[i - 1]:]
                del stack[-plan[i - 1]:]
                stack.append(ex.submit(run_merge, take, ev))
                merges.append(len(take))
                del take
        if len(stack) > 1:
            ev = torch.cuda.Event()
            ev.record(s_main)
            merges.append(len(stack))
            stack = [ex.submit(run_merge, list(stack), ev)]
        C = stack[0].result() if isinstance(stack[0], Future) else stack[0]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) * 1e3
    t_mrg = acct["t_mrg"]
    frac = (t_exp + t_mrg - wall) / t_mrg if t_mrg > 0 else 0.0
    return C, dict(t_expand_ms=t_exp, t_merge_ms=t_mrg, peak_list_bytes=acct["peak"], partial_nnz=sizes,
                   merges=merges, nnz=C.nnz, wall_ms=wall, overlap=True, overlap_frac=frac,
                   merge_calls=calls)


def batched_mcl(A: "mcl.DeviceCSC", comp_ptr: torch.Tensor, params=None, tol: float = 1e-9,
                max_iter: int = 100):
    """Iterate every component until its change drops below `tol` (Alg. 1's
    loop, per component); converged components are frozen (copied) by the
    library.  Returns (A_final, iterations per component, info); info
    ["converged"] flags the components whose change fell below `tol` within
    `max_iter` iterations and info["not_converged"] counts the others."""
    ncomp = comp_ptr.numel() - 1
    active = torch.ones(ncomp, dtype=torch.uint8, device=comp_ptr.device)
    iters = np.zeros(ncomp, np.int64)
    converged = np.zeros(ncomp, bool)
    steps = []
    it = 0
    while it < max_iter:
        t = time.perf_counter()
        A, change, st = mcl.iterate(A, params, comp_ptr=comp_ptr, active=active)
        steps.append(dict(ms=(time.perf_counter() - t) * 1e3, active=int(active.sum()), flops=st["flops"]))
        act = active.cpu().numpy().astype(bool)
        iters[act] += 1
        converged |= act & (change < tol)
        still = act & (change >= tol)
        it += 1
        if not still.any():
            break
        active = torch.from_numpy(still.astype(np.uint8)).to(comp_ptr.device)
    return A, iters, dict(calls=it, steps=steps, converged=converged,
                          not_converged=int((~converged).sum()))


def component_block(W, c0: int, c1: int):
    """Host CSC of the diagonal block [c0, c1) of a block-diagonal matrix, rows renumbered."""
    from mclgen import CSC
    p0, p1 = int(W.colptr[c0]), int(W.colptr[c1])
    return CSC(c1 - c0, c1 - c0, (W.colptr[c0:c1 + 1] - p0).astype(np.int64),
               (W.rowidx[p0:p1] - c0).astype(np.int32), W.val[p0:p1].copy())


def component_mcl(Ablk: "mcl.DeviceCSC", params=None, tol: float = 1e-9, max_iter: int = 100):
    """Plain loop on one component: iterate until the change drops below
    `tol`.  Returns (A_final, iterations, converged) -- converged is False
    when `max_iter` iterations ended with the change still >= `tol`."""
    it = 0
    converged = False
    while it < max_iter:
        Ablk, change, _ = mcl.iterate(Ablk, params)
        it += 1
        if change < tol:
            converged = True
            break
    return Ablk, it, converged


def same_block(Abig: "mcl.DeviceCSC", c0: int, c1: int, Ablk: "mcl.DeviceCSC") -> bool:
    """Is the diagonal block [c0, c1) of Abig (all its columns' entries lie in
    the block) bit-identical to Ablk?"""
    p0, p1 = int(Abig.colptr[c0]), int(Abig.colptr[c1])
    cp = Abig.colptr[c0:c1 + 1] - p0
    return (torch.equal(cp, Ablk.colptr) and torch.equal(Abig.rowidx[p0:p1] - c0, Ablk.rowidx)
            and torch.equal(Abig.val[p0:p1], Ablk.val))


def save_checkpoint(path: str, A: "mcl.DeviceCSC", iteration: int, converged: bool = False):
    """Writes the iterate, the number of iterations done and whether the run
    has converged to `path` (numpy .npz): first to a temporary file next to
    it, then renamed over it, so an interrupted run never leaves a partial
    checkpoint."""
    import os
    tmp = path + ".tmp.npz"
    np.savez(tmp, nrows=A.nrows, ncols=A.ncols, iteration=iteration, converged=converged,
             colptr=A.colptr.cpu().numpy(), rowidx=A.rowidx.cpu().numpy(), val=A.val.cpu().numpy())
    os.replace(tmp, path)


def load_checkpoint(path: str):
    """(iterate on the device, iterations done, converged) from
    save_checkpoint's file."""
    with np.load(path, allow_pickle=False) as z:
        A = mcl.DeviceCSC(int(z["nrows"]), int(z["ncols"]), torch.from_numpy(z["colptr"]).cuda(),
                          torch.from_numpy(z["rowidx"]).cuda(), torch.from_numpy(z["val"]).cuda())
        return A, int(z["iteration"]), bool(z["converged"])


def run_mcl(A: "mcl.DeviceCSC", params=None, tol: float = 1e-9, max_iter: int = 100, log_path: str = None,
            checkpoint_path: str = None, checkpoint_every: int = 1, resume: bool = False):
    """Alg. 1 on the GPU from a column-stochastic A: iterate until the change
    drops below `tol` (or `max_iter` iterations in all), then label the
    connected components of the final pattern.  Returns (A_final,
    iterations, labels, ncomp, converged); labels is a device int32 tensor
    (smallest vertex id of each vertex's cluster).

    log_path: one JSON line per iteration is appended (iteration, change,
    flops, product and kept nnz, overflowed and HBM-table columns, phases,
    milliseconds).  checkpoint_path: every `checkpoint_every` iterations the
    iterate and the iteration count are saved there; with resume=True a run
    starts from that checkpoint when it exists (A is then not used) and ends
    bit-identical to an uninterrupted run."""
    import json
    import os
    it = 0
    converged = False
    if resume and checkpoint_path and os.path.exists(checkpoint_path):
        A, it, converged = load_checkpoint(checkpoint_path)
    logf = open(log_path, "a") if log_path else None
    try:
        while it < max_iter and not converged:
            A, change, st = mcl.iterate(A, params, iteration=it)
            it += 1
            if logf:
                logf.write(json.dumps({"iteration": it, "change": change, "flops": st["flops"],
                                       "nnz_product": st["nnz_product"], "nnz_kept": st["nnz_kept"],
                                       "n_overflow": st["n_overflow"], "n_global": st["n_global"],
                                       "n_phases": st["n_phases"], "t_total_ms": round(st["t_total_ms"], 3)})
                           + "\n")
                logf.flush()
            if change < tol:
                converged = True
            if checkpoint_path and (converged or it % max(1, checkpoint_every) == 0 or it == max_iter):
                save_checkpoint(checkpoint_path, A, it, converged)
    finally:
        if logf:
            logf.close()
    labels, ncomp = mcl.components(A)
    return A, it, labels, ncomp, converged
