"""Planted-cluster similarity graphs (the synthetic stand-in for the protein
networks of the paper's evaluation, Table 1), emitted as sorted CSC.

Recipe (one seeded ``numpy`` PCG64 stream per graph):

1. Cluster sizes are drawn i.i.d. from the discrete power law
   p(s) ~ s**-alpha on [s_min, s_cap] (inverse CDF), then rescaled by
   largest-remainder rounding so that they sum to the vertex count, never
   below s_min.
2. Vertex ids are randomly permuted (globally, or inside each component for
   block-diagonal multi-component graphs), so clusters have no id locality.
3. Every unordered intra-cluster pair is an edge with probability p_in
   (geometric skipping over the cluster's pair space, one SplitMix64 stream
   per cluster, in ``gen.c``), weight U(0.5, 1).
4. round(x / (1 - x) * m_in) inter-cluster pairs are added with endpoints
   uniform in different clusters (of the same component), weight in (0, 0.3];
   duplicate pairs keep their first draw.
5. The matrix is symmetrised and every column receives a self-loop whose
   weight is the column's largest off-diagonal weight (1.0 when the vertex is
   isolated).

Values are *not* normalised: making the matrix column stochastic is the first
step of the clustering method itself and is done by each consumer.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import ctypes
import os
import subprocess
import threading

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "gen.c")
_GEN_LIB = os.path.join(_HERE, "libmclgen.so")
_gen = None
_gen_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the sampling / assembly helper (gcc, OpenMP)."""
    if force or not os.path.exists(_GEN_LIB):
        tmp = _GEN_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _GEN_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _genlib():
    global _gen
    with _gen_lock:
        if _gen is None:
            if not os.path.exists(_GEN_LIB):
                build(force=False)
            lib = ctypes.CDLL(_GEN_LIB)
            vp, i64 = ctypes.c_void_p, ctypes.c_int64
            lib.gen_intra.argtypes = [i64, vp, vp, vp, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp]
            lib.gen_assemble.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
            _gen = lib
    return _gen


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclasses.dataclass
class CSC:
    """Host CSC matrix: int64 colptr (ncols+1), int32 rowidx, float64 val."""

    nrows: int
    ncols: int
    colptr: np.ndarray
    rowidx: np.ndarray
    val: np.ndarray
    labels: np.ndarray | None = None      # planted cluster id per vertex
    comp_ptr: np.ndarray | None = None    # component vertex ranges (int64)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_scipy(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.val, self.rowidx.astype(np.int64), self.colptr),
                             shape=(self.nrows, self.ncols))

    @staticmethod
    def from_scipy(m, **kw) -> "CSC":
        m = sp.csc_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return CSC(m.shape[0], m.shape[1], m.indptr.astype(np.int64),
                   m.indices.astype(np.int32), m.data.astype(np.float64), **kw)

    def column(self, j: int):
        a, b = self.colptr[j], self.colptr[j + 1]
        return self.rowidx[a:b], self.val[a:b]

    def restrict_columns(self, cols) -> "CSC":
        """The sub-matrix made of the listed columns (all rows)."""
        cols = np.asarray(cols, np.int64)
        cnt = self.colptr[cols + 1] - self.colptr[cols]
        cp = np.zeros(len(cols) + 1, np.int64)
        cp[1:] = np.cumsum(cnt)
        if len(cols):
            starts = np.repeat(self.colptr[cols], cnt)
            within = np.arange(int(cp[-1]), dtype=np.int64) - np.repeat(cp[:-1], cnt)
            idx = starts + within
        else:
            idx = np.zeros(0, np.int64)
        return CSC(self.nrows, len(cols), cp, self.rowidx[idx], self.val[idx])


# --------------------------------------------------------------------------
# cluster sizes
# --------------------------------------------------------------------------

def powerlaw_sizes(u: np.ndarray, alpha: float, s_min: int, s_cap: int) -> np.ndarray:
    """Map uniforms u in [0,1) to sizes of the discrete power law on [s_min, s_cap]."""
    s = np.arange(s_min, s_cap + 1, dtype=np.float64)
    pdf = s ** (-alpha)
    cdf = np.cumsum(pdf)
    cdf /= cdf[-1]
    idx = np.searchsorted(cdf, u, side="right")
    return (s_min + np.minimum(idx, len(s) - 1)).astype(np.int64)


def _rescale_to_total(sizes: np.ndarray, total: int, s_min: int) -> np.ndarray:
    """Largest-remainder rescale of ``sizes`` to sum exactly ``total`` (each >= s_min)."""
    k = len(sizes)
    if k * s_min > total:
        raise ValueError("too many clusters for the vertex count")
    f = sizes.astype(np.float64) * (total / float(sizes.sum()))
    base = np.floor(f).astype(np.int64)
    rem = total - int(base.sum())
    if rem > 0:
        order = np.argsort(-(f - base), kind="stable")
        base[order[:rem]] += 1
    base = np.maximum(base, s_min)
    excess = int(base.sum()) - total
    while excess > 0:                 # take the clamp excess back from the largest
        order = np.argsort(-base, kind="stable")
        for i in order:
            take = min(excess, int(base[i]) - s_min)
            if take > 0:
                base[i] -= take
                excess -= take
            if excess == 0:
                break
    return base


def _rescale_groups(sizes: np.ndarray, group: np.ndarray, totals: np.ndarray, s_min) -> np.ndarray:
    """Vectorised largest-remainder rescale of every group of ``sizes`` (group
    ids ascending, contiguous) to sum to totals[group]; each size >= s_min[group]
    where possible (the clamp excess is taken from the group's largest)."""
    sizes = sizes.astype(np.float64)
    ng = len(totals)
    gsum = np.bincount(group, weights=sizes, minlength=ng)
    f = sizes * (totals / gsum)[group]
    base = np.floor(f).astype(np.int64)
    rem = totals - np.bincount(group, weights=base, minlength=ng).astype(np.int64)
    order = np.lexsort((-(f - base), group))
    start = np.zeros(ng + 1, np.int64)
    start[1:] = np.cumsum(np.bincount(group, minlength=ng))
    rank = np.empty(len(sizes), np.int64)
    rank[order] = np.arange(len(sizes)) - start[group[order]]
    base += (rank < rem[group]).astype(np.int64)
    smin = np.broadcast_to(np.asarray(s_min), (ng,))[group]
    base = np.maximum(base, smin)
    excess = np.bincount(group, weights=base, minlength=ng).astype(np.int64) - totals
    if (excess > 0).any():
        big = np.lexsort((-base, group))          # largest first within each group
        first = big[start[:-1][start[:-1] < start[1:]]]
        gi = group[first]
        base[first] -= np.maximum(excess[gi], 0)
    return base


def _expected_nnz_per_col(sizes, n, p_in, x):
    m_in = p_in * float(np.sum(sizes * (sizes - 1) / 2.0))
    m_x = x / (1.0 - x) * m_in
    return (2.0 * (m_in + m_x) + n) / n


def fit_cap_for_density(u, n, alpha, s_min, target_nnz_per_col, p_in=0.3, x=0.05,
                        lo=None, hi=200000):
    """Bisection on s_cap so that the expected nnz/col of the rescaled sizes hits
    the target (the same uniforms ``u`` are reused for every trial cap)."""
    lo = lo or s_min + 1

    def dens(cap):
        s = _rescale_to_total(powerlaw_sizes(u, alpha, s_min, cap), n, s_min)
        return _expected_nnz_per_col(s, n, p_in, x)

    if dens(hi) < target_nnz_per_col:
        return hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if dens(mid) < target_nnz_per_col:
            lo = mid
        else:
            hi = mid
    return hi


# --------------------------------------------------------------------------
# edge sampling helpers
# --------------------------------------------------------------------------

def _bernoulli_positions(rng, total: int, p: float) -> np.ndarray:
    """Positions in [0, total) selected independently with probability p
    (geometric skipping)."""
    if total <= 0 or p <= 0:
        return np.zeros(0, np.int64)
    if p >= 1:
        return np.arange(total, dtype=np.int64)
    out = []
    pos = -1
    while True:
        need = int(p * (total - pos) + 6 * math.sqrt(total * p) + 64)
        gaps = rng.geometric(p, size=need).astype(np.int64)
        cs = pos + np.cumsum(gaps)
        keep = cs[cs < total]
        out.append(keep)
        if len(keep) < len(cs):
            break
        pos = int(cs[-1])
    return np.concatenate(out)


def _tri_decode(q: np.ndarray, s: np.ndarray):
    """Row-major strict upper triangle index q of an s x s matrix -> (a, b), a < b."""
    qf = q.astype(np.float64)
    sf = s.astype(np.float64)
    t = 2.0 * sf - 1.0
    a = np.floor((t - np.sqrt(np.maximum(t * t - 8.0 * qf, 0.0))) / 2.0).astype(np.int64)
    a = np.clip(a, 0, np.maximum(s - 2, 0))

    def off(a_):
        return a_ * (2 * s - a_ - 1) // 2

    for _ in range(3):
        up = off(a + 1) <= q
        a = np.where(up & (a + 1 <= s - 2), a + 1, a)
        down = off(a) > q
        a = np.where(down, a - 1, a)
    b = q - off(a) + a + 1
    return a, b


def _assemble(n, ei, ej, ew, labels, comp_ptr=None) -> CSC:
    """Symmetrise the undirected edge list, add self-loops, emit sorted CSC."""
    lib = _genlib()
    ei = np.ascontiguousarray(ei, np.int32)
    ej = np.ascontiguousarray(ej, np.int32)
    ew = np.ascontiguousarray(ew, np.float64)
    E = len(ei)
    colptr = np.empty(n + 1, np.int64)
    rowidx = np.empty(2 * E + n, np.int32)
    val = np.empty(2 * E + n, np.float64)
    lib.gen_assemble(n, E, _ptr(ei), _ptr(ej), _ptr(ew), _ptr(colptr), _ptr(rowidx), _ptr(val))
    return CSC(n, n, colptr, rowidx, val, labels=labels, comp_ptr=comp_ptr)


def _intra_edges(sizes, cstart, perm, p_in, seed, w_in):
    """Intra-cluster pairs with probability p_in (per-cluster streams)."""
    lib = _genlib()
    sizes = np.ascontiguousarray(sizes, np.int64)
    cstart = np.ascontiguousarray(cstart, np.int64)
    perm = np.ascontiguousarray(perm, np.int64)
    ncl = len(sizes)
    counts = np.zeros(ncl, np.int64)
    lib.gen_intra(ncl, _ptr(sizes), _ptr(cstart), _ptr(perm), float(p_in), int(seed) & (2**64 - 1),
                  float(w_in[0]), float(w_in[1]), _ptr(counts), None, None, None, None)
    offs = np.zeros(ncl + 1, np.int64)
    offs[1:] = np.cumsum(counts)
    E = int(offs[-1])
    u = np.empty(E, np.int32)
    v = np.empty(E, np.int32)
    w = np.empty(E, np.float64)
    lib.gen_intra(ncl, _ptr(sizes), _ptr(cstart), _ptr(perm), float(p_in), int(seed) & (2**64 - 1),
                  float(w_in[0]), float(w_in[1]), _ptr(counts), _ptr(offs), _ptr(u), _ptr(v), _ptr(w))
    return u, v, w, counts


# --------------------------------------------------------------------------
# planted graphs
# --------------------------------------------------------------------------

def planted_components(comp_sizes: Sequence[int], comp_clusters: Sequence[int], *,
                       alpha=2.0, s_min=3, s_cap=2000, p_in=0.3, x=0.05,
                       w_in=(0.5, 1.0), w_x=0.3, seed=0, permute="within",
                       rng=None) -> CSC:
    """Block-diagonal union of planted-cluster components.

    Component c occupies the contiguous vertex range comp_ptr[c]:comp_ptr[c+1];
    ids are permuted inside each component (``permute="within"``) or over the
    whole graph (``permute="global"``, single-component graphs only)."""
    rng = rng or np.random.Generator(np.random.PCG64(seed))
    comp_sizes = np.asarray(comp_sizes, np.int64)
    comp_clusters = np.asarray(comp_clusters, np.int64)
    ncomp = len(comp_sizes)
    n = int(comp_sizes.sum())
    comp_ptr = np.zeros(ncomp + 1, np.int64)
    comp_ptr[1:] = np.cumsum(comp_sizes)

    # 1. cluster sizes per component (one shared power law, rescaled per component)
    ccomp = np.repeat(np.arange(ncomp), comp_clusters)
    smin_c = np.maximum(1, np.minimum(s_min, comp_sizes // np.maximum(comp_clusters, 1)))
    u = rng.random(len(ccomp))
    raw = powerlaw_sizes(u, alpha, s_min, max(s_cap, s_min + 1))
    sizes = _rescale_groups(raw, ccomp, comp_sizes, smin_c)
    cstart = np.zeros(len(sizes) + 1, np.int64)
    cstart[1:] = np.cumsum(sizes)          # cluster ranges in position space
    pos_cluster = np.repeat(np.arange(len(sizes)), sizes)

    # 2. permutation position -> vertex id
    if permute == "global":
        perm = rng.permutation(n).astype(np.int64)
    else:
        key = rng.random(n)
        pos_comp = np.repeat(np.arange(ncomp), comp_sizes)
        perm = np.lexsort((key, pos_comp)).astype(np.int64)
        # perm currently sorts positions; invert to map position -> id inside comp
        inv = np.empty(n, np.int64)
        inv[perm] = np.arange(n)
        perm = inv
    labels = np.empty(n, np.int32)
    labels[perm] = pos_cluster.astype(np.int32)

    # 3. intra-cluster edges
    ei, ej, ew, per_cluster = _intra_edges(sizes, cstart[:-1], perm, p_in,
                                           int(rng.integers(0, 2**63)), w_in)

    # 4. inter-cluster edges, per component
    m_in_c = np.bincount(ccomp, weights=per_cluster, minlength=ncomp).astype(np.float64)
    ncl_c = np.bincount(ccomp, minlength=ncomp)
    m_x_c = np.where(ncl_c > 1, np.rint(x / (1.0 - x) * m_in_c), 0).astype(np.int64)
    xc = np.repeat(np.arange(ncomp), m_x_c)
    lo = comp_ptr[xc]
    span = comp_sizes[xc]
    u = lo + (rng.random(len(xc)) * span).astype(np.int64)
    v = lo + (rng.random(len(xc)) * span).astype(np.int64)
    idx = np.nonzero(pos_cluster[u] == pos_cluster[v])[0]
    while len(idx):
        v[idx] = lo[idx] + (rng.random(len(idx)) * span[idx]).astype(np.int64)
        idx = idx[pos_cluster[u[idx]] == pos_cluster[v[idx]]]
    wx = w_x * (1.0 - rng.random(len(xc)))      # in (0, w_x]
    xu, xv = perm[u], perm[v]
    lo_v, hi_v = np.minimum(xu, xv), np.maximum(xu, xv)
    keyx = lo_v * n + hi_v
    _, first = np.unique(keyx, return_index=True)
    first.sort()
    ei = np.concatenate([ei, lo_v[first].astype(np.int32)])
    ej = np.concatenate([ej, hi_v[first].astype(np.int32)])
    ew = np.concatenate([ew, wx[first]])
    return _assemble(n, ei, ej, ew, labels, comp_ptr)


def planted_graph(n, n_clusters, *, alpha=2.0, s_min=3, s_cap=2000, p_in=0.3, x=0.05,
                  seed=0, **kw) -> CSC:
    """Single-component planted graph with globally permuted ids."""
    return planted_components([n], [n_clusters], alpha=alpha, s_min=s_min, s_cap=s_cap,
                              p_in=p_in, x=x, seed=seed, permute="global", **kw)


#: s_cap that gives ~100 nnz/col for 1,000,000 vertices in 50,000 clusters
#: (alpha 2, s_min 3); fixed by ``fit_cap_for_density`` with seed 1001.
def _config1_cap(seed=1001, n=1_000_000, k=50_000, target=100.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(k)
    return fit_cap_for_density(u, n, 2.0, 3, target)


def config0_graph(seed=1000, s_cap=None) -> CSC:
    """10,000 vertices in 400 power-law clusters (alpha 2, min 3)."""
    if s_cap is None:
        s_cap = 2100
    return planted_graph(10_000, 400, s_cap=s_cap, seed=seed)


def config1_graph(seed=1001, n=1_000_000, n_clusters=50_000, target_nnz_per_col=100.0,
                  s_cap=None) -> CSC:
    """n vertices in power-law clusters with s_cap fitted for ~100 nnz/col."""
    if s_cap is None:
        rng = np.random.Generator(np.random.PCG64(seed + 7919))
        u = rng.random(n_clusters)
        s_cap = fit_cap_for_density(u, n, 2.0, 3, target_nnz_per_col)
    return planted_graph(n, n_clusters, s_cap=s_cap, seed=seed)


def config3_graph(seed=1003, n_comp=20_000, total=4_000_000, smin_comp=8, smax_comp=30_000,
                  target_nnz_per_col=80.0, alpha_comp=None, s_cap=None) -> CSC:
    """Block-diagonal union of ``n_comp`` planted components with power-law sizes
    in [smin_comp, smax_comp]; each gets max(1, round(size/25)) clusters."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_comp)
    if alpha_comp is None:               # fit the exponent so the sizes sum ~ total
        lo, hi = 1.01, 3.0
        for _ in range(40):
            mid = 0.5 * (lo + hi)
            s = powerlaw_sizes(u, mid, smin_comp, smax_comp).sum()
            if s > total:
                lo = mid
            else:
                hi = mid
        alpha_comp = 0.5 * (lo + hi)
    csz = powerlaw_sizes(u, alpha_comp, smin_comp, smax_comp)
    ccl = np.maximum(1, np.rint(csz / 25.0)).astype(np.int64)
    if s_cap is None:
        u2 = np.random.Generator(np.random.PCG64(seed + 7919)).random(int(ccl.sum()))
        grp = np.repeat(np.arange(n_comp), ccl)
        smin_c = np.maximum(1, np.minimum(3, csz // ccl))
        lo, hi = 4, 30000
        while hi - lo > 1:
            mid = (lo + hi) // 2
            sizes = _rescale_groups(powerlaw_sizes(u2, 2.0, 3, mid), grp, csz, smin_c)
            d = _expected_nnz_per_col(sizes, int(csz.sum()), 0.3, 0.05)
            if d < target_nnz_per_col:
                lo = mid
            else:
                hi = mid
        s_cap = hi
    return planted_components(csz, ccl, alpha=2.0, s_min=3, s_cap=s_cap, seed=seed + 1,
                              permute="within")


# --------------------------------------------------------------------------
# small structured / random inputs for tests
# --------------------------------------------------------------------------

def random_csc(nrows, ncols, mean_nnz_per_col, seed=0, skew=0.0, empty_frac=0.0) -> CSC:
    """Random positive CSC; per-column counts are Poisson (or lognormal-skewed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if skew > 0:
        lam = mean_nnz_per_col * rng.lognormal(0.0, skew, ncols) / math.exp(skew * skew / 2)
    else:
        lam = np.full(ncols, float(mean_nnz_per_col))
    cnt = np.minimum(rng.poisson(lam), nrows).astype(np.int64)
    if empty_frac > 0:
        cnt[rng.random(ncols) < empty_frac] = 0
    colptr = np.zeros(ncols + 1, np.int64)
    colptr[1:] = np.cumsum(cnt)
    rows = np.empty(int(colptr[-1]), np.int32)
    for j in range(ncols):
        c = int(cnt[j])
        if c:
            if c * 4 < nrows:
                r = np.unique(rng.integers(0, nrows, size=2 * c + 8))
                r = rng.permutation(r)[:c] if len(r) >= c else rng.choice(nrows, c, replace=False)
            else:
                r = rng.choice(nrows, c, replace=False)
            rows[colptr[j]:colptr[j + 1]] = np.sort(r)
    val = 1e-3 + rng.random(len(rows))
    return CSC(nrows, ncols, colptr, rows, val)


def random_symmetric_graph(n, p, seed=0) -> CSC:
    """Erdos-Renyi-style symmetric weighted graph with self-loops (tiny tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    w = 0.05 + rng.random(int(keep.sum()))
    return _assemble(n, iu[keep], ju[keep], w, np.zeros(n, np.int32))


def clique_union(sizes: Sequence[int], w=1.0, seed=None) -> CSC:
    """Disjoint complete graphs with uniform weight w (self-loops weight w)."""
    n = int(sum(sizes))
    ei, ej = [], []
    off = 0
    labels = np.empty(n, np.int32)
    for c, s in enumerate(sizes):
        iu, ju = np.triu_indices(s, 1)
        ei.append(iu + off)
        ej.append(ju + off)
        labels[off:off + s] = c
        off += s
    ei = np.concatenate(ei) if ei else np.zeros(0, np.int64)
    ej = np.concatenate(ej) if ej else np.zeros(0, np.int64)
    if seed is not None:
        perm = np.random.Generator(np.random.PCG64(seed)).permutation(n)
        ei, ej = perm[ei], perm[ej]
        lab = np.empty(n, np.int32)
        lab[perm] = labels
        labels = lab
    return _assemble(n, ei, ej, np.full(len(ei), float(w)), labels)


def two_triangles() -> CSC:
    """Triangles {0,1,2} and {3,4,5} joined by the single edge 2-3."""
    ei = np.array([0, 0, 1, 3, 3, 4, 2])
    ej = np.array([1, 2, 2, 4, 5, 5, 3])
    w = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.2])
    return _assemble(6, ei, ej, w, np.array([0, 0, 0, 1, 1, 1], np.int32))


# --------------------------------------------------------------------------
# one process's share of a 2D block distribution (Sparse SUMMA stages)
# --------------------------------------------------------------------------

def stripe_blocks(N=10_000_000, grid=8, row_stripe=0, col_stripe=1, target_nnz_per_col=480.0,
                  alpha=2.0, s_min=3, p_in=0.3, x=0.05, seed=1002, scale=None, workers=8):
    """Blocks A[row_stripe, k] and A[k, col_stripe] (k = 0..grid-1) of one
    planted graph on N vertices, generated block by block without building the
    rest of the graph.

    Unordered block pairs {I, K} are drawn once from their own RNG stream and
    A[K, I] is the transpose of A[I, K], so the blocks are consistent with one
    symmetric graph.  Global column sums are not available to a single block
    row/column, so every weight is multiplied by ``scale`` (default
    1/target_nnz_per_col, the magnitude of a column-normalised entry); diagonal
    blocks get unit self-loops.  Blocks are generated by `workers` threads
    (the result does not depend on it).  Returns (A_row: list of CSC, A_col:
    list of CSC).
    """
    base = np.random.Generator(np.random.PCG64(seed))
    n_clusters = max(1, int(round(N / 21.6)))
    u = base.random(n_clusters)
    cap = fit_cap_for_density(u, N, alpha, s_min, target_nnz_per_col, p_in, x)
    sizes = _rescale_to_total(powerlaw_sizes(u, alpha, s_min, cap), N, s_min)
    perm = base.permutation(N).astype(np.int64)
    pos_cluster = np.repeat(np.arange(len(sizes)), sizes)
    vcl = np.empty(N, np.int64)
    vcl[perm] = pos_cluster
    bs = N // grid
    if scale is None:
        scale = 1.0 / target_nnz_per_col
    m_in_total = p_in * float(np.sum(sizes * (sizes - 1) / 2.0))
    m_x_total = x / (1.0 - x) * m_in_total

    # members of every cluster inside every stripe, sorted by (cluster, id)
    order = np.lexsort((np.arange(N), vcl))
    seg = {}

    def members(I):
        if I not in seg:
            sel = order[(order // bs) == I]
            cl = vcl[sel]
            cnt = np.bincount(cl, minlength=len(sizes)).astype(np.int64)
            ptr = np.zeros(len(sizes) + 1, np.int64)
            ptr[1:] = np.cumsum(cnt)
            seg[I] = (sel, cnt, ptr)
        return seg[I]

    cache = {}

    def gen_block(key):
        if True:
            a_, b_ = key
            rng = np.random.Generator(np.random.PCG64([seed, a_, b_]))
            selA, cntA, ptrA = members(a_)
            selB, cntB, ptrB = members(b_)
            if a_ == b_:
                P = cntA * (cntA - 1) // 2
            else:
                P = cntA * cntB
            Pc = np.zeros(len(P) + 1, np.int64)
            Pc[1:] = np.cumsum(P)
            q = _bernoulli_positions(rng, int(Pc[-1]), p_in)
            cl = np.searchsorted(Pc, q, side="right") - 1
            ql = q - Pc[cl]
            if a_ == b_:
                ia, ib = _tri_decode(ql, cntA[cl])
                gu, gv = selA[ptrA[cl] + ia], selA[ptrA[cl] + ib]
            else:
                ia, ib = ql // cntB[cl], ql % cntB[cl]
                gu, gv = selA[ptrA[cl] + ia], selB[ptrB[cl] + ib]
            w = 0.5 + 0.5 * rng.random(len(q))
            # inter-cluster pairs falling in this block
            frac = (bs * bs * (1.0 if a_ != b_ else 0.5)) / (N * (N - 1) / 2.0)
            mx = rng.poisson(m_x_total * frac)
            xu = a_ * bs + rng.integers(0, bs, mx)
            xv = b_ * bs + rng.integers(0, bs, mx)
            ok = (vcl[xu] != vcl[xv]) & (xu != xv)
            xu, xv = xu[ok], xv[ok]
            wx = 0.3 * (1.0 - rng.random(len(xu)))
            kk = np.minimum(xu, xv) * N + np.maximum(xu, xv)
            _, first = np.unique(kk, return_index=True)
            first.sort()
            gu = np.concatenate([gu, xu[first]])
            gv = np.concatenate([gv, xv[first]])
            w = np.concatenate([w, wx[first]]) * scale
            r = (gu - a_ * bs).astype(np.int32)
            c = (gv - b_ * bs).astype(np.int32)
            if a_ == b_:
                rr = np.concatenate([r, c, np.arange(bs, dtype=np.int32)])
                cc = np.concatenate([c, r, np.arange(bs, dtype=np.int32)])
                ww = np.concatenate([w, w, np.full(bs, scale)])
            else:
                rr, cc, ww = r, c, w
            m = sp.csc_matrix((ww, (rr, cc)), shape=(bs, bs))
            m.sum_duplicates()
            m.sort_indices()
            return m

    # every block pair once (each from its own RNG stream), several at a time
    keys = sorted({(min(row_stripe, k), max(row_stripe, k)) for k in range(grid)}
                  | {(min(k, col_stripe), max(k, col_stripe)) for k in range(grid)})
    for I in sorted({i for kk in keys for i in kk}):
        members(I)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(workers, len(keys)))) as ex:
        cache = dict(zip(keys, ex.map(gen_block, keys)))

    def block(I, K):
        key = (min(I, K), max(I, K))
        m = cache[key]
        if (I, K) != (min(I, K), max(I, K)):
            m = m.T.tocsc()
            m.sort_indices()
        return CSC.from_scipy(m)

    A_row = [block(row_stripe, k) for k in range(grid)]
    A_col = [block(k, col_stripe) for k in range(grid)]
    return A_row, A_col
