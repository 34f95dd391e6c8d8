"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
dense brute force, a library sparse product, closed forms, invariants and
textbook special cases.  No GPU needed."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import dense
from mclgen import (CSC, clique_union, random_csc, random_symmetric_graph, two_triangles,
                    planted_graph)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def to_dense(M: CSC) -> np.ndarray:
    return M.to_scipy().toarray()


def pattern(M: CSC) -> np.ndarray:
    D = np.zeros((M.nrows, M.ncols), bool)
    for j in range(M.ncols):
        D[M.rowidx[M.colptr[j]:M.colptr[j + 1]], j] = True
    return D


# ---------------------------------------------------------------- expansion

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_expand_matches_dense_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n, m, p = 150, 120, 90
    A = random_csc(n, m, 6, seed=seed, skew=0.8)
    B = random_csc(m, p, 5, seed=seed + 100, skew=0.8, empty_frac=0.05)
    C, flops, nnz = oracle.expand(A, B)
    Ad, Bd = to_dense(A), to_dense(B)
    assert np.array_equal(pattern(C), dense.pattern_product(Ad, Bd))
    assert np.array_equal(flops, dense.flops(Ad, Bd))
    assert np.array_equal(nnz, dense.pattern_product(Ad, Bd).sum(axis=0))
    ref = Ad @ Bd
    got = to_dense(C)
    assert np.allclose(got, ref, rtol=1e-14, atol=0)
    # rows ascending and unique within each column
    for j in range(C.ncols):
        r = C.rowidx[C.colptr[j]:C.colptr[j + 1]]
        assert np.all(np.diff(r) > 0)
    del rng


def test_expand_matches_scipy_product():
    W = planted_graph(8000, 300, s_cap=400, seed=5)
    A = oracle.normalize(W)
    C, flops, _ = oracle.expand(A, A)
    S = (A.to_scipy() @ A.to_scipy()).tocsc()
    S.sort_indices()
    assert np.array_equal(C.colptr, S.indptr)
    assert np.array_equal(C.rowidx, S.indices)
    assert np.allclose(C.val, S.data, rtol=1e-13, atol=0)
    assert flops.sum() == int(np.diff(A.colptr)[A.rowidx].sum())


def test_product_of_stochastic_is_stochastic():
    A = oracle.normalize(planted_graph(3000, 120, s_cap=300, seed=9))
    s0 = np.add.reduceat(A.val, A.colptr[:-1])
    assert np.allclose(s0, 1.0, atol=4 * 64 * 2.0 ** -53)
    C, _, _ = oracle.expand(A, A)
    s = np.add.reduceat(C.val, C.colptr[:-1])
    assert np.allclose(s, 1.0, atol=1e-13)


def test_expand_empty_and_rectangular():
    A = random_csc(40, 30, 0.0, seed=1)          # all columns empty
    B = random_csc(30, 20, 3, seed=2)
    C, flops, nnz = oracle.expand(A, B)
    assert C.nnz == 0 and flops.sum() == 0
    A = random_csc(40, 30, 4, seed=3)
    C, _, _ = oracle.expand(A, B)
    assert (C.nrows, C.ncols) == (40, 20)
    assert np.allclose(to_dense(C), to_dense(A) @ to_dense(B), rtol=1e-14, atol=0)


# ---------------------------------------------------------------- prune

def _product(seed, n=180, deg=10):
    A = oracle.normalize(random_symmetric_graph(n, deg / n, seed=seed))
    B, _, _ = oracle.expand(A, A)
    return B


@pytest.mark.parametrize("seed,S,R,theta", [(0, 20, 30, 1.2e-2), (1, 50, 70, 1e-2),
                                            (2, 40, 10, 1e-4), (3, 5, 0, 1e-2),
                                            (4, 0, 50, 1.2e-2), (6, 20, 30, 1e-3)])
def test_prune_matches_dense_sort(seed, S, R, theta):
    B = _product(seed)
    C, info = oracle.prune(B, theta=theta, select=S, recover=R, pct=0.9)
    Bd = to_dense(B)
    Bp = pattern(B)
    keep = pattern(C)
    for j in range(B.ncols):
        k, t, mode = dense.prune_column(Bd[:, j], Bp[:, j], theta, S, R, 0.9)
        mB, mP = info["mass"][j], info["mass_above"][j]
        near = abs(mP - 0.9 * mB) <= 1e-12 * mB
        if not near:
            assert mode == info["mode"][j], j
            assert np.array_equal(k, keep[:, j]), j
    assert np.allclose(to_dense(C)[keep], Bd[keep], rtol=0, atol=0)


def test_prune_identity_special_case():
    B = _product(7)
    C, info = oracle.prune(B, theta=0.0, select=0, recover=0)
    assert np.array_equal(C.colptr, B.colptr) and np.array_equal(C.rowidx, B.rowidx)
    assert np.array_equal(C.val, B.val)


def test_prune_uniform_column_kept_whole():
    # one column of 50 equal values, select 10: ties at the 10th value are all kept
    m = 50
    B = CSC(100, 1, np.array([0, m], np.int64), np.arange(0, 2 * m, 2, dtype=np.int32),
            np.full(m, 0.02))
    C, info = oracle.prune(B, theta=1e-4, select=10, recover=0)
    assert C.nnz == m and info["mode"][0] == 2


def test_prune_properties():
    B = _product(11, n=300, deg=14)
    R, S = 40, 25
    C, info = oracle.prune(B, theta=1e-2, select=S, recover=R)
    assert (info["mode"] == 1).sum() > 100
    for j in range(B.ncols):
        r0, v0 = B.column(j)
        r1, v1 = C.column(j)
        dropped = np.setdiff1d(r0, r1)
        if len(r1) and len(dropped):
            assert v1.min() >= v0[np.isin(r0, dropped)].max()
        if info["mode"][j] == 1:
            assert len(r1) >= min(R, len(r0))
        if info["mode"][j] == 2:
            assert len(r1) >= S


# ---------------------------------------------------------------- inflation

def test_inflate_r1_is_identity_on_stochastic():
    A = oracle.normalize(random_symmetric_graph(200, 0.05, seed=3))
    I = oracle.inflate(A, 1.0)
    assert np.allclose(I.val, A.val, rtol=1e-15 * 8, atol=0)


def test_inflate_uniform_stays_uniform_and_sums_to_one():
    A = oracle.normalize(clique_union([4, 9, 30]))
    I = oracle.inflate(A, 2.0)
    assert np.allclose(I.val, A.val, rtol=4e-16, atol=0)
    B = _product(5)
    I = oracle.inflate(B, 2.0)
    s = np.add.reduceat(I.val, I.colptr[:-1])
    assert np.allclose(s, 1.0, atol=1e-14)
    Id = to_dense(I)
    Bd = to_dense(B)
    j = 3
    nz = Bd[:, j] != 0
    assert np.allclose(Id[nz, j], Bd[nz, j] ** 2 / (Bd[nz, j] ** 2).sum(), rtol=1e-14)


# ---------------------------------------------------------------- whole iterations

def test_disjoint_cliques_are_a_fixed_point():
    sizes = [3, 5, 17, 64, 250]
    W = clique_union(sizes, w=1.0, seed=4)
    A0 = oracle.normalize(W)
    A1, info = oracle.iterate(A0)
    assert np.array_equal(A1.rowidx, A0.rowidx)
    assert np.allclose(A1.val, A0.val, rtol=1e-15 * 4, atol=0)
    assert info["delta"].max() < 1e-9
    A, it, lab = oracle.mcl(W)
    assert it == 1
    # clusters = cliques (labels are min vertex ids)
    _, truth = np.unique(W.labels, return_inverse=True)
    _, got = np.unique(lab, return_inverse=True)
    assert len(np.unique(got)) == len(sizes)
    for c in range(len(sizes)):
        assert len(np.unique(got[truth == c])) == 1


def test_two_triangles_two_clusters():
    A, it, lab = oracle.mcl(two_triangles())
    assert len(np.unique(lab)) == 2
    assert lab[0] == lab[1] == lab[2] == 0 and lab[3] == lab[4] == lab[5] == 3


def test_block_diagonal_independence():
    g1 = planted_graph(300, 12, s_cap=80, seed=1)
    g2 = planted_graph(200, 8, s_cap=80, seed=2)
    U = CSC.from_scipy(sp.block_diag([g1.to_scipy(), g2.to_scipy()]))
    a1, _ = oracle.iterate(oracle.normalize(g1), select=30, recover=40)
    a2, _ = oracle.iterate(oracle.normalize(g2), select=30, recover=40)
    au, _ = oracle.iterate(oracle.normalize(U), select=30, recover=40)
    both = CSC.from_scipy(sp.block_diag([a1.to_scipy(), a2.to_scipy()]))
    assert np.array_equal(au.rowidx, both.rowidx)
    assert np.array_equal(au.val, both.val)          # bit-exact


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_iteration_matches_dense_mcl(seed):
    n = 40 + 4 * seed
    W = random_symmetric_graph(n, 0.12, seed=seed)
    S, R, theta = 6, 9, 1e-3
    A = oracle.normalize(W)
    Wd = to_dense(W)
    assert np.allclose(to_dense(A), dense.normalize(Wd), rtol=1e-15, atol=0)
    for _ in range(6):       # compare step by step from the same input
        An, info = oracle.iterate(A, theta=theta, select=S, recover=R, pct=0.9)
        Ad = to_dense(A)
        B = Ad @ Ad
        Bp = dense.pattern_product(Ad, Ad)
        C, keep, modes = dense.prune(B, Bp, theta, S, R, 0.9)
        ref = dense.inflate(C, keep, 2.0)
        assert np.array_equal(pattern(An), keep)
        assert np.allclose(to_dense(An), ref, rtol=1e-13, atol=0)
        A = An
    # full runs give the same clusters
    _, it, lab = oracle.mcl(W, theta=theta, select=S, recover=R)
    _, _, itd, labd = dense.mcl(Wd, theta=theta, S=S, R=R)
    assert np.array_equal(lab, labd) and it == itd


def test_clusters_are_min_id_components():
    W = random_symmetric_graph(60, 0.03, seed=8)
    lab = oracle.clusters(W)
    assert np.array_equal(lab, dense.components(to_dense(W) != 0))


# ---------------------------------------------------------------- Cohen estimator

def test_cohen_keys_are_unit_exponential():
    keys = np.array([oracle.cohen_key(7, 0, i, l, 5) for i in range(4000) for l in range(5)])
    assert keys.min() > 0
    assert abs(keys.mean() - 1.0) < 0.03            # ~4 standard errors
    assert abs((keys > 1.0).mean() - np.exp(-1)) < 0.015


def test_cohen_estimator_mean_and_spread():
    # column 0 reaches rows 0..n0-1 through two middle vertices; column 1 reaches one row
    n0 = 300
    A = CSC(n0, 3, np.array([0, 150, n0, n0 + 1], np.int64),
            np.concatenate([np.arange(n0), [5]]).astype(np.int32), np.ones(n0 + 1))
    B = CSC(3, 3, np.array([0, 2, 3, 3], np.int64), np.array([0, 1, 2], np.int32), np.ones(3))
    for r, sd_expected in ((5, 1 / np.sqrt(3)), (10, 1 / np.sqrt(8))):
        est = np.array([oracle.cohen_estimate(A, B, r=r, seed=3, it=t) for t in range(3000)])
        e0 = est[:, 0] / n0
        assert abs(e0.mean() - 1.0) < 4 * sd_expected / np.sqrt(3000)
        assert abs(e0.std() / sd_expected - 1.0) < 0.15
        assert np.all(est[:, 2] == 0.0)              # empty column
        # a single reached row: est = (r-1) / sum of that row's r keys
        t = 17
        ref = (r - 1) / sum(oracle.cohen_key(3, t, 5, l, r) for l in range(r))
        assert est[t, 1] == pytest.approx(ref, rel=1e-15)


def test_cohen_exact_when_reaching_all_rows_is_unbiased_on_planted():
    A = oracle.normalize(planted_graph(4000, 150, s_cap=200, seed=2))
    _, _, nnz = oracle.expand(A, A)
    est = np.mean([oracle.cohen_estimate(A, A, r=5, seed=1, it=t) for t in range(40)], axis=0)
    big = nnz > 50
    assert abs(np.median(est[big] / nnz[big]) - 1.0) < 0.08


# ---------------------------------------------------------------- merging (Section 4)

def test_alg2_schedule_matches_hand_trace():
    rows = np.loadtxt(os.path.join(GOLDEN, "alg2_schedule_8.txt"), dtype=np.int64)
    groups, depth = oracle.binary_merge_schedule(8)
    assert groups == list(rows[:, 1])
    assert depth == 1


def test_immediate_merge_closed_form():
    rows = np.loadtxt(os.path.join(GOLDEN, "merge_closed_forms.txt"), dtype=np.int64)
    for k, n, ops in rows:
        # k-1 successive two-way merges of disjoint length-n lists into the running result
        cost, acc = 0, n
        for _ in range(k - 1):
            cost += acc + n
            acc += n
        assert cost == ops == n * (k * (k + 1) // 2 - 1)


def test_merged_partials_equal_direct_product():
    k = 8
    rng = np.random.default_rng(0)
    A = random_csc(300, 8 * 40, 5, seed=1, skew=0.5)
    B = random_csc(8 * 40, 250, 6, seed=2, skew=0.5)
    parts = []
    for s in range(k):
        As = CSC.from_scipy(A.to_scipy()[:, s * 40:(s + 1) * 40])
        Bs = CSC.from_scipy(B.to_scipy()[s * 40:(s + 1) * 40, :])
        parts.append(oracle.expand(As, Bs)[0])
    direct, _, _ = oracle.expand(A, B)
    multi = oracle.merge(parts)
    binm, peak = oracle.binary_merge(parts)
    for M in (multi, binm):
        assert np.array_equal(M.colptr, direct.colptr)
        assert np.array_equal(M.rowidx, direct.rowidx)
        assert np.allclose(M.val, direct.val, rtol=1e-12, atol=0)
    # multiway holds every partial at once; binary merge never more than that
    assert peak <= sum(p.nnz for p in parts)
    del rng


def test_merge_heap_sums_in_list_order():
    a = CSC(4, 1, np.array([0, 2], np.int64), np.array([0, 2], np.int32), np.array([1e16, 1.0]))
    b = CSC(4, 1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([1.0]))
    c = CSC(4, 1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([-1e16]))
    m = oracle.merge([a, b, c])
    assert m.val[0] == (1e16 + 1.0) + -1e16


# ---------------------------------------------------------------- change between iterates

def _csc_cols(nrows, cols):
    """CSC from a list of {row: value} dicts (one per column)."""
    colptr = [0]
    rows, vals = [], []
    for c in cols:
        for r in sorted(c):
            rows.append(r)
            vals.append(c[r])
        colptr.append(len(rows))
    return CSC(nrows, len(cols), np.array(colptr, np.int64), np.array(rows, np.int32),
               np.array(vals, np.float64))


def test_delta_hand_worked_union_of_patterns():
    """Alg. 1 loops while the iterate changes; the change is the largest
    |a_new - a_old| over the union of both patterns (an entry present on one
    side only counts with its full value).  Dyadic values make every
    difference exact."""
    old = _csc_cols(6, [
        {0: 0.5, 2: 0.5},            # max on an old-only entry (row 2): 0.5
        {0: 0.875, 1: 0.125},        # max on a new-only entry (row 3): 0.375
        {1: 0.5, 2: 0.5},            # disjoint patterns: 0.75
        {4: 0.25, 5: 0.75},          # identical: 0
        {},                          # empty old column, new has one entry: 1
        {3: 1.0},                    # new column empty: 1
        {0: 0.25, 1: 0.25, 2: 0.5},  # max on a shared entry: 0.25
    ])
    new = _csc_cols(6, [
        {0: 0.625, 1: 0.375},
        {0: 0.5625, 1: 0.0625, 3: 0.375},
        {0: 0.25, 3: 0.75},
        {4: 0.25, 5: 0.75},
        {5: 1.0},
        {},
        {0: 0.5, 1: 0.125, 2: 0.375},
    ])
    want = np.array([0.5, 0.375, 0.75, 0.0, 1.0, 1.0, 0.25])
    got = oracle.delta(old, new)
    assert np.array_equal(got, want), (got, want)
    # the change is symmetric in its two arguments
    assert np.array_equal(oracle.delta(new, old), want)
