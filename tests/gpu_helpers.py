"""Comparison helpers for the GPU parity tests (host side only)."""
from __future__ import annotations

import numpy as np

from mclgen import CSC

TIE_RTOL = 1e-12


def csc_columns_equal(g: CSC, o: CSC):
    """Boolean per column: identical row patterns."""
    n = o.ncols
    if np.array_equal(g.colptr, o.colptr) and np.array_equal(g.rowidx, o.rowidx):
        return np.ones(n, bool)
    eq = np.zeros(n, bool)
    for j in range(n):
        a0, a1 = g.colptr[j], g.colptr[j + 1]
        b0, b1 = o.colptr[j], o.colptr[j + 1]
        eq[j] = (a1 - a0 == b1 - b0) and np.array_equal(g.rowidx[a0:a1], o.rowidx[b0:b1])
    return eq


def max_rel_diff_on_equal_columns(g: CSC, o: CSC, eq):
    worst = 0.0
    if eq.all() and np.array_equal(g.colptr, o.colptr):
        d = np.abs(g.val - o.val) / np.maximum(np.abs(o.val), 1e-300)
        return float(d.max(initial=0.0))
    for j in np.nonzero(eq)[0]:
        a0, a1 = g.colptr[j], g.colptr[j + 1]
        b0, b1 = o.colptr[j], o.colptr[j + 1]
        if a1 > a0:
            d = np.abs(g.val[a0:a1] - o.val[b0:b1]) / np.maximum(np.abs(o.val[b0:b1]), 1e-300)
            worst = max(worst, float(d.max()))
    return worst


def tie_explains(j, B: CSC, g: CSC, o: CSC, info, theta, pct):
    """A column whose GPU and oracle kept sets differ is acceptable only if the
    difference is a near-tie: the recovery test sum(P) < pct*sum(B) is within
    1e-12 of equality, or every differing entry is within 1e-12 (relative) of
    the column threshold or of theta."""
    mB, mP = info["mass"][j], info["mass_above"][j]
    if abs(mP - pct * mB) <= TIE_RTOL * mB:
        return True
    t = info["threshold"][j]
    r0, v0 = B.column(j)
    gr = set(g.rowidx[g.colptr[j]:g.colptr[j + 1]].tolist())
    orr = set(o.rowidx[o.colptr[j]:o.colptr[j + 1]].tolist())
    diff = gr.symmetric_difference(orr)
    vals = {int(r): float(v) for r, v in zip(r0, v0)}
    for r in diff:
        v = vals.get(int(r))
        if v is None:
            return False
        if not (abs(v - t) <= TIE_RTOL * max(t, 1e-300) or abs(v - theta) <= TIE_RTOL * theta):
            return False
    return True


def restrict_columns(M: CSC, cols) -> CSC:
    """Sub-matrix of the listed columns (all rows)."""
    return M.restrict_columns(cols)
