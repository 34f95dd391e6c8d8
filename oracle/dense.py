"""Dense numpy brute-force MCL for tiny graphs -- TEST INFRASTRUCTURE.

An independent second implementation used to pin the C oracle: dense
matrices, numpy's matrix product and per-column numpy sorts, no sparse data
structures.  It follows the same readings of the paper as the C oracle
(Alg. 1 steps; recovery/selection rules; ties kept; renormalisation after the
Hadamard power; convergence on the max entry change).
"""
from __future__ import annotations

import numpy as np


def normalize(W: np.ndarray) -> np.ndarray:
    s = W.sum(axis=0)
    return np.divide(W, s, out=np.zeros_like(W), where=s > 0)


def expand(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    return A @ B


def pattern_product(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Boolean pattern of A B (exact, integer arithmetic)."""
    return ((A != 0).astype(np.int64) @ (B != 0).astype(np.int64)) > 0


def flops(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """flops_j = sum over nonzero b_kj of nnz(A_*k)."""
    nnzA = (A != 0).sum(axis=0)
    return ((B != 0) * nnzA[:, None]).sum(axis=0)


def prune_column(b: np.ndarray, pattern: np.ndarray, theta, S, R, pct):
    """Returns (kept mask, threshold, mode) for one dense column; ``pattern``
    marks the structurally nonzero entries."""
    vals = b[pattern]
    above = vals >= theta
    nP = int(above.sum())
    mP = vals[above].sum()
    mB = vals.sum()
    m = len(vals)
    srt = np.sort(vals)[::-1]
    if R > 0 and nP < R and mP < pct * mB:
        t = srt[R - 1] if m >= R else 0.0
        mode = 1
    elif S > 0 and nP > S:
        t = srt[S - 1]
        mode = 2
    else:
        t = theta
        mode = 0
    return pattern & (b >= t), t, mode


def prune(B: np.ndarray, Bpat: np.ndarray, theta=1e-4, S=1100, R=1400, pct=0.9):
    keep = np.zeros_like(Bpat)
    modes = np.zeros(B.shape[1], np.int32)
    for j in range(B.shape[1]):
        keep[:, j], _, modes[j] = prune_column(B[:, j], Bpat[:, j], theta, S, R, pct)
    return np.where(keep, B, 0.0), keep, modes


def inflate(C: np.ndarray, pat: np.ndarray, r=2.0) -> np.ndarray:
    P = np.where(pat, C ** r, 0.0)
    s = P.sum(axis=0)
    return np.divide(P, s, out=np.zeros_like(P), where=s > 0)


def components(pat: np.ndarray) -> np.ndarray:
    """Weakly connected components by repeated label propagation; min-id labels."""
    n = pat.shape[0]
    sym = pat | pat.T
    lab = np.arange(n)
    while True:
        nb = np.where(sym, lab[None, :], n).min(axis=1)
        new = np.minimum(lab, nb)
        if np.array_equal(new, lab):
            return lab
        lab = new


def mcl(W: np.ndarray, theta=1e-4, S=1100, R=1400, pct=0.9, r=2.0, tol=1e-9, max_iter=100):
    A = normalize(W)
    pat = A != 0
    it = 0
    for it in range(1, max_iter + 1):
        B = A @ A
        Bpat = pattern_product(pat.astype(float), pat.astype(float))
        C, keep, _ = prune(B, Bpat, theta, S, R, pct)
        An = inflate(C, keep, r)
        d = np.abs(An - A).max() if A.size else 0.0
        A, pat = An, keep
        if d < tol:
            break
    return A, pat, it, components(pat)
