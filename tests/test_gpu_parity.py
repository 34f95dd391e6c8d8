"""GPU parity: every C-ABI entry point against the CPU oracle on the same
seeded inputs (sizes that span many LDS bins, ragged tails and empty
columns).  Expansion values must be bit-identical (same FMA order); pruned
patterns identical except documented near-ties; inflated values within
1e-12 relative."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from mclgen import (CSC, clique_union, config0_graph, planted_graph, random_csc,
                    random_symmetric_graph, planted_components)
from gpu_helpers import (csc_columns_equal, max_rel_diff_on_equal_columns, restrict_columns,
                         tie_explains)
from paper_2002_10083_amd.tuning import VARIANTS as _NV

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def up(m, M):
    return m.DeviceCSC.from_host(M)


def assert_same_matrix(g: CSC, o: CSC, exact=True, rtol=0.0):
    assert np.array_equal(g.colptr, o.colptr)
    assert np.array_equal(g.rowidx, o.rowidx)
    if exact:
        assert np.array_equal(g.val, o.val)
    else:
        d = np.abs(g.val - o.val) / np.maximum(np.abs(o.val), 1e-300)
        assert float(d.max(initial=0.0)) <= rtol


# ---------------------------------------------------------------- expansion

@pytest.mark.parametrize("case", ["rect", "skew", "empty", "planted", "dense_cols", "bigcluster"])
def test_expand_bit_exact(mcl, case):
    print("case", case, flush=True)
    if case == "rect":
        A = random_csc(3000, 2000, 12, seed=1)
        B = random_csc(2000, 1500, 9, seed=2, empty_frac=0.05)
    elif case == "skew":
        A = random_csc(5000, 5000, 20, seed=3, skew=1.2)
        B = random_csc(5000, 3000, 15, seed=4, skew=1.2)
    elif case == "empty":
        A = random_csc(100, 80, 0.0, seed=5)
        B = random_csc(80, 60, 3, seed=6)
    elif case == "planted":
        A = oracle.normalize(planted_graph(6000, 200, s_cap=600, seed=7))
        B = A
    elif case == "bigcluster":   # product columns up to ~6000 rows: the largest LDS bins
        A = oracle.normalize(planted_graph(40000, 2000, s_cap=2100, seed=70))
        B = A
    else:  # a few very long columns -> large tables / HBM-table path
        A = random_csc(40000, 600, 400, seed=8)
        B = random_csc(600, 64, 300, seed=9)
    C, flops, nnz = oracle.expand(A, B)
    G, st = mcl.expand(up(mcl, A), up(mcl, B), estimator=mcl.EST_BOUND)
    assert_same_matrix(G.to_host(), C, exact=True)
    assert st["flops"] == int(flops.sum())
    assert st["nnz_product"] == C.nnz


def test_expand_identical_across_estimators_and_forced_overflow(mcl):
    A = oracle.normalize(planted_graph(8000, 250, s_cap=900, seed=11))
    dA = up(mcl, A)
    ref, _ = mcl.expand(dA, dA, estimator=mcl.EST_BOUND)
    coh, s1 = mcl.expand(dA, dA, estimator=mcl.EST_COHEN, seed=5)
    ovf, s2 = mcl.expand(dA, dA, estimator=mcl.EST_COHEN, est_scale=0.01)
    assert s2["n_overflow"] > 0
    for X in (coh, ovf):
        assert torch.equal(X.colptr, ref.colptr)
        assert torch.equal(X.rowidx, ref.rowidx)
        assert torch.equal(X.val, ref.val)
    C, _, _ = oracle.expand(A, A)
    assert_same_matrix(ovf.to_host(), C, exact=True)


def test_symbolic_flops_and_exact_nnz(mcl):
    A = oracle.normalize(planted_graph(5000, 180, s_cap=700, seed=12))
    _, flops, nnz = oracle.expand(A, A)
    f, z = mcl.symbolic(up(mcl, A), up(mcl, A), exact=True)
    assert np.array_equal(f.cpu().numpy(), flops)
    assert np.array_equal(z.cpu().numpy(), nnz)


def test_cohen_estimate_matches_oracle(mcl):
    A = oracle.normalize(planted_graph(4000, 150, s_cap=400, seed=13))
    for r in (2, 3, 5, 10, 12, 16):  # every padded key stride (4, 8, 12, 16)
        ref = oracle.cohen_estimate(A, A, r=r, seed=77, it=3)
        est = mcl.estimate(up(mcl, A), up(mcl, A), estimator=mcl.EST_COHEN, cohen_keys=r, seed=77,
                           iteration=3).cpu().numpy()
        assert np.allclose(est, ref, rtol=2e-6, atol=0)


# ---------------------------------------------------------------- prune / inflate

@pytest.mark.parametrize("S,R,theta", [(1100, 1400, 1e-4), (40, 60, 1e-3), (25, 0, 2e-3),
                                       (0, 80, 5e-3), (0, 0, 1e-4)])
def test_prune_parity(mcl, S, R, theta):
    A = oracle.normalize(planted_graph(6000, 200, s_cap=800, seed=14))
    B, _, _ = oracle.expand(A, A)
    O, info = oracle.prune(B, theta=theta, select=S, recover=R, pct=0.9)
    G, st = mcl.prune(up(mcl, B), prune_threshold=theta, select_num=S, recover_num=R)
    g = G.to_host()
    eq = csc_columns_equal(g, O)
    for j in np.nonzero(~eq)[0]:
        assert tie_explains(j, B, g, O, info, theta, 0.9), j
    assert max_rel_diff_on_equal_columns(g, O, eq) == 0.0   # kept values are copies
    assert st["n_selected"] == int((info["mode"] == 2).sum())
    assert st["n_recovered"] == int((info["mode"] == 1).sum())


def test_prune_exact_ties(mcl):
    """Select / recover thresholds that fall on tied values: every tie is kept
    (columns with <= 64 and > 64 tied candidates, values differing only in the
    last bit, and a recovery column of equal sub-threshold values)."""
    x = 0.25
    xu = float(np.nextafter(x, 1.0))
    cols = [np.full(50, 0.02),                                    # select, 50 tied
            np.full(100, 0.01),                                   # select, 100 tied
            np.concatenate([0.5 + 1e-3 * np.arange(5), np.full(40, 0.003)]),
            np.array([xu, x] * 10),                               # 10th largest = x + 1 ulp
            np.full(200, 1e-5)]                                   # recover, 200 tied
    colptr = np.zeros(len(cols) + 1, np.int64)
    rows, vals = [], []
    for j, c in enumerate(cols):
        colptr[j + 1] = colptr[j] + len(c)
        rows.append(np.arange(0, 2 * len(c), 2, dtype=np.int32))
        vals.append(c.astype(np.float64))
    B = CSC(400, len(cols), colptr, np.concatenate(rows), np.concatenate(vals))
    O, info = oracle.prune(B, theta=1e-4, select=10, recover=80, pct=0.9)
    assert list(info["mode"]) == [2, 2, 2, 2, 1]
    assert list(np.diff(O.colptr)) == [50, 100, 45, 10, 200]
    G, st = mcl.prune(up(mcl, B), prune_threshold=1e-4, select_num=10, recover_num=80)
    assert_same_matrix(G.to_host(), O, exact=True)


def test_inflate_parity(mcl):
    A = oracle.normalize(planted_graph(5000, 160, s_cap=500, seed=15))
    B, _, _ = oracle.expand(A, A)
    for r in (2.0, 1.5, 3.0):
        O = oracle.inflate(B, r)
        G = up(mcl, B)
        err = mcl.inflate_(G, r)
        g = G.to_host()
        assert np.array_equal(g.rowidx, O.rowidx)
        d = np.abs(g.val - O.val) / O.val
        assert d.max() <= 1e-12
        assert err <= 1e-13


def test_normalize_parity(mcl):
    W = planted_graph(3000, 100, s_cap=300, seed=16)
    O = oracle.normalize(W)
    G = up(mcl, W)
    mcl.normalize_(G)
    d = np.abs(G.to_host().val - O.val) / O.val
    assert d.max() <= 1e-13


# ---------------------------------------------------------------- fused iteration

def check_iterate(mcl, A, theta=1e-4, S=1100, R=1400, **kw):
    An_o, info = oracle.iterate(A, theta=theta, select=S, recover=R, pct=0.9)
    G, change, st = mcl.iterate(up(mcl, A), prune_threshold=theta, select_num=S, recover_num=R, **kw)
    g = G.to_host()
    eq = csc_columns_equal(g, An_o)
    B = info["B"]
    for j in np.nonzero(~eq)[0]:
        assert tie_explains(j, B, g, An_o, info, theta, 0.9), j
    assert max_rel_diff_on_equal_columns(g, An_o, eq) <= 1e-12
    if eq.all():
        assert abs(change - info["delta"].max()) <= 1e-12 * max(1.0, info["delta"].max())
    assert st["flops"] == int(info["flops"].sum())
    assert st["nnz_product"] == int(info["nnz_product"].sum())
    return G, change, st


@pytest.mark.parametrize("seed", [0, 1])
def test_iterate_parity_config0(mcl, seed):
    A = oracle.normalize(config0_graph(seed=1000 + seed))
    check_iterate(mcl, A)


@pytest.mark.parametrize("S,R,theta", [(40, 60, 1e-3), (20, 0, 5e-3), (0, 100, 1e-2)])
def test_iterate_parity_small_k(mcl, S, R, theta):
    A = oracle.normalize(planted_graph(5000, 180, s_cap=500, seed=17))
    check_iterate(mcl, A, theta=theta, S=S, R=R)


# policy v uses variant min(v, count - 1) in every bin: together they cover
# every launch shape of every bin
ALL_VARIANTS = [sum(min(v, nv - 1) << (4 * b) for b, nv in enumerate(_NV)) for v in range(max(_NV))]


def test_launch_variants_are_bit_identical(mcl):
    A = oracle.normalize(planted_graph(40000, 2000, s_cap=2100, seed=71))
    dA = up(mcl, A)
    ref, c0, st0 = mcl.iterate(dA, bin_policy=0)
    assert max(st0["bin_cols"][4:7]) > 0
    E0, _ = mcl.expand(dA, dA, bin_policy=0)
    for pol in ALL_VARIANTS[1:]:
        X, c1, _ = mcl.iterate(dA, bin_policy=pol)
        assert torch.equal(X.rowidx, ref.rowidx) and torch.equal(X.val, ref.val) and c1 == c0
        E1, _ = mcl.expand(dA, dA, bin_policy=pol)
        assert torch.equal(E1.rowidx, E0.rowidx) and torch.equal(E1.val, E0.val)


@pytest.mark.parametrize("S,R,theta", [(40, 60, 1e-3), (20, 0, 5e-3), (0, 100, 1e-2), (300, 2500, 2e-3)])
def test_iterate_parity_split_bins_prune_branches(mcl, S, R, theta):
    """Columns of the split bins (4-6) and of the multi-pass bin decide their
    prune branch before sorting (selection, threshold, and recovery decided
    from the unsorted column sums); every branch must match the oracle."""
    A = oracle.normalize(planted_graph(40000, 2000, s_cap=2100, seed=73))
    _, _, st = check_iterate(mcl, A, theta=theta, S=S, R=R)
    assert max(st["bin_cols"][4:7]) > 0
    if R > 0:
        assert st["n_recovered"] > 0
    if S > 0:
        assert st["n_selected"] > 0


def test_iterate_parity_big_clusters(mcl):
    A = oracle.normalize(planted_graph(40000, 2000, s_cap=2100, seed=72))
    _, _, st = check_iterate(mcl, A)
    assert st["bin_cols"][6] > 0


def test_iterate_is_composition_of_exports(mcl):
    A = oracle.normalize(planted_graph(6000, 200, s_cap=700, seed=18))
    dA = up(mcl, A)
    F, _, _ = mcl.iterate(dA, select_num=50, recover_num=80, prune_threshold=1e-3)
    B, _ = mcl.expand(dA, dA)
    C, _ = mcl.prune(B, select_num=50, recover_num=80, prune_threshold=1e-3)
    mcl.inflate_(C, 2.0)
    assert torch.equal(F.colptr, C.colptr) and torch.equal(F.rowidx, C.rowidx)
    assert torch.equal(F.val, C.val)


def test_iterate_identical_across_estimators(mcl):
    A = oracle.normalize(planted_graph(8000, 250, s_cap=900, seed=19))
    dA = up(mcl, A)
    ref, c0, _ = mcl.iterate(dA, estimator=mcl.EST_BOUND)
    for kw in (dict(estimator=mcl.EST_COHEN, seed=3), dict(estimator=mcl.EST_COHEN, est_scale=0.02)):
        X, c1, _ = mcl.iterate(dA, **kw)
        assert torch.equal(X.rowidx, ref.rowidx) and torch.equal(X.val, ref.val) and c1 == c0


def test_mcl_to_convergence_matches_oracle(mcl):
    W = config0_graph()
    Ao, it_o, lab_o = oracle.mcl(W)
    A = up(mcl, W)
    mcl.normalize_(A)
    it = 0
    for it in range(1, 101):
        A, change, _ = mcl.iterate(A, iteration=it)
        if change < 1e-9:
            break
    lab = oracle.clusters(A.to_host())
    assert np.array_equal(lab, lab_o)
    assert abs(it - it_o) <= 1


def test_clique_fixed_point(mcl):
    W = clique_union([3, 7, 31, 200, 1100], seed=2)
    A0 = oracle.normalize(W)
    G, change, _ = mcl.iterate(up(mcl, A0))
    assert change < 1e-9
    g = G.to_host()
    assert np.array_equal(g.rowidx, A0.rowidx)
    assert np.allclose(g.val, A0.val, rtol=4e-16 * 8, atol=0)


# ---------------------------------------------------------------- batched form

def test_batched_iterate_equals_per_component(mcl):
    U = planted_components([300, 40, 2000, 8, 900, 1500], [12, 2, 80, 1, 36, 60], s_cap=300, seed=21)
    A = oracle.normalize(U)
    dA = up(mcl, A)
    comp = torch.from_numpy(U.comp_ptr).cuda()
    ncomp = len(U.comp_ptr) - 1
    active = torch.tensor([1, 1, 0, 1, 1, 0], dtype=torch.uint8, device="cuda")
    G, change, st = mcl.iterate(dA, comp_ptr=comp, active=active)
    g = G.to_host()
    full, _, _ = mcl.iterate(dA)
    f = full.to_host()
    for c in range(ncomp):
        lo, hi = U.comp_ptr[c], U.comp_ptr[c + 1]
        src = f if active[c] else A
        a0, a1 = g.colptr[lo], g.colptr[hi]
        b0, b1 = src.colptr[lo], src.colptr[hi]
        assert np.array_equal(g.rowidx[a0:a1], src.rowidx[b0:b1])
        assert np.array_equal(g.val[a0:a1], src.val[b0:b1])
        if not active[c]:
            assert change[c] == 0.0
    # a component iterated alone gives the same bytes as inside the batch
    c = 4
    lo, hi = U.comp_ptr[c], U.comp_ptr[c + 1]
    sub = CSC.from_scipy(A.to_scipy()[lo:hi, lo:hi])
    S1, ch1, _ = mcl.iterate(up(mcl, sub))
    s1 = S1.to_host()
    a0, a1 = g.colptr[lo], g.colptr[hi]
    assert np.array_equal(s1.rowidx + lo, g.rowidx[a0:a1])
    assert np.array_equal(s1.val, g.val[a0:a1])
    assert ch1 == change[c]


# ---------------------------------------------------------------- merge

def test_merge_partials_parity(mcl):
    k = 8
    A = random_csc(4000, 8 * 500, 6, seed=31, skew=0.6)
    B = random_csc(8 * 500, 3000, 7, seed=32, skew=0.6)
    parts = []
    for s in range(k):
        As = CSC.from_scipy(A.to_scipy()[:, s * 500:(s + 1) * 500])
        Bs = CSC.from_scipy(B.to_scipy()[s * 500:(s + 1) * 500, :])
        parts.append(oracle.expand(As, Bs)[0])
    M_o = oracle.merge(parts)
    G, st = mcl.merge_partials([up(mcl, p) for p in parts])
    assert_same_matrix(G.to_host(), M_o, exact=True)
    direct, _, _ = oracle.expand(A, B)
    assert_same_matrix(G.to_host(), direct, exact=False, rtol=1e-12)
    # groups of the binary-merge schedule give the oracle's grouped sums
    g12, _ = mcl.merge_partials([up(mcl, parts[0]), up(mcl, parts[1])])
    assert_same_matrix(g12.to_host(), oracle.merge(parts[:2]), exact=True)


def _random_parts(nparts, nrows, ncols, col_len, seed):
    """nparts matrices with sorted, unique rows per column; column j of every
    part draws col_len(j) rows from a shared pool, so rows repeat across parts."""
    rng = np.random.default_rng(seed)
    parts = []
    for p in range(nparts):
        colptr = [0]
        rows, vals = [], []
        for j in range(ncols):
            m = min(col_len(j), nrows)
            r = np.sort(rng.choice(nrows, size=m, replace=False)).astype(np.int32)
            rows.append(r)
            vals.append(rng.random(m) + 0.01)
            colptr.append(colptr[-1] + m)
        parts.append(CSC(nrows, ncols, np.array(colptr, np.int64), np.concatenate(rows),
                         np.concatenate(vals)))
    return parts


def test_merge_large_columns_and_empty_columns(mcl):
    # columns from 1 to 12,000 merged entries (several LDS bins and the HBM
    # table); column 3 is empty in every part
    sizes = {0: 3000, 1: 1100, 2: 40, 3: 0, 4: 1025, 5: 2500, 6: 1}
    parts = _random_parts(4, 6000, 7, lambda j: sizes[j], seed=91)
    assert max(sum(int(np.diff(p.colptr)[j]) for p in parts) for j in range(7)) > 8192
    G, _ = mcl.merge_partials([up(mcl, p) for p in parts])
    assert_same_matrix(G.to_host(), oracle.merge(parts), exact=True)


def test_merge_many_parts(mcl):
    # many parts, and the first 32 of them
    parts = _random_parts(40, 500, 60, lambda j: 5 + (7 * j) % 40, seed=92)
    G, _ = mcl.merge_partials([up(mcl, p) for p in parts])
    assert_same_matrix(G.to_host(), oracle.merge(parts), exact=True)
    G2, _ = mcl.merge_partials([up(mcl, p) for p in parts[:32]])
    assert_same_matrix(G2.to_host(), oracle.merge(parts[:32]), exact=True)


# ---------------------------------------------------------------- errors

def test_invalid_input_is_rejected(mcl):
    A = random_csc(50, 50, 4, seed=41)
    bad = CSC(A.nrows, A.ncols, A.colptr.copy(), A.rowidx.copy(), A.val.copy())
    j = int(np.argmax(np.diff(bad.colptr) >= 2))
    s = bad.colptr[j]
    bad.rowidx[s], bad.rowidx[s + 1] = bad.rowidx[s + 1], bad.rowidx[s]   # unsorted column
    with pytest.raises(mcl.MclError) as e:
        mcl.expand(up(mcl, bad), up(mcl, A), validate=1)
    assert e.value.code == mcl.MCL_EINVAL
    with pytest.raises(mcl.MclError) as e:
        mcl.expand(up(mcl, A), up(mcl, random_csc(40, 10, 2, seed=1)))
    assert e.value.code == mcl.MCL_EINVAL
    neg = CSC(A.nrows, A.ncols, A.colptr, A.rowidx, -A.val)
    with pytest.raises(mcl.MclError):
        mcl.iterate(up(mcl, neg), validate=1)


def test_allocator_failure_releases_everything(mcl):
    A = oracle.normalize(planted_graph(2000, 80, s_cap=200, seed=42))
    dA = up(mcl, A)
    al = mcl._allocator()
    for n_ok in (0, 3, 9):
        al.fail_after = al.count + n_ok
        with pytest.raises(mcl.MclError) as e:
            mcl.iterate(dA)
        assert e.value.code == mcl.MCL_ENOMEM
        al.fail_after = None
        torch.cuda.synchronize()
        assert len(al.live) == 0
    G, _, _ = mcl.iterate(dA)     # still usable afterwards
    assert G.nnz > 0


def test_phased_iterate_is_identical(mcl):
    A = oracle.normalize(planted_graph(8000, 250, s_cap=900, seed=23))
    dA = up(mcl, A)
    ref, c0, st0 = mcl.iterate(dA, phase_bytes=-1)
    assert st0["n_phases"] == 1
    for pb in (3 << 20, 400 << 10):
        X, c1, st = mcl.iterate(dA, phase_bytes=pb)
        assert st["n_phases"] > 1
        assert torch.equal(X.colptr, ref.colptr) and torch.equal(X.rowidx, ref.rowidx)
        assert torch.equal(X.val, ref.val) and c1 == c0
        assert st["nnz_product"] == st0["nnz_product"] and st["flops"] == st0["flops"]


def test_phased_batched_iterate_is_identical(mcl):
    U = planted_components([300, 40, 2000, 8, 900, 1500], [12, 2, 80, 1, 36, 60], s_cap=300, seed=24)
    dA = up(mcl, oracle.normalize(U))
    comp = torch.from_numpy(U.comp_ptr).cuda()
    active = torch.tensor([1, 0, 1, 1, 0, 1], dtype=torch.uint8, device="cuda")
    ref, c0, _ = mcl.iterate(dA, comp_ptr=comp, active=active, phase_bytes=-1)
    X, c1, st = mcl.iterate(dA, comp_ptr=comp, active=active, phase_bytes=256 << 10)
    assert st["n_phases"] > 1
    assert torch.equal(X.colptr, ref.colptr) and torch.equal(X.rowidx, ref.rowidx)
    assert torch.equal(X.val, ref.val) and np.array_equal(c0, c1)


def _huge_cluster_graph():
    # clusters of ~4,200, ~8,300 and ~11,500 vertices, no inter-cluster edges:
    # product columns of up to ~11,500 rows, beyond the largest LDS table set
    return oracle.normalize(planted_graph(24000, 3, s_cap=13000, p_in=0.03, x=0.0, seed=61))


def test_multipass_columns_iterate_parity(mcl):
    A = _huge_cluster_graph()
    _, _, st = check_iterate(mcl, A)
    assert st["bin_cols"][7] > 0


def test_multipass_columns_expand_and_exact_path(mcl):
    A = _huge_cluster_graph()
    C, flops, nnz = oracle.expand(A, A)
    dA = up(mcl, A)
    G, st = mcl.expand(dA, dA)
    assert st["bin_cols"][7] > 0
    assert_same_matrix(G.to_host(), C, exact=True)
    # underestimated sizes: overflow, exact count, HBM tables -- same result
    X, st2 = mcl.expand(dA, dA, est_scale=0.5)
    assert st2["n_overflow"] > 0
    assert torch.equal(X.rowidx, G.rowidx) and torch.equal(X.val, G.val)
    ref, _, _ = mcl.iterate(dA)
    Y, _, st3 = mcl.iterate(dA, est_scale=0.5)
    assert torch.equal(Y.rowidx, ref.rowidx) and torch.equal(Y.val, ref.val)


def _hub_graph(n=30000, hubs=300, hub_len=400, seed=81):
    """Column `hubs` references every hub column 0..hubs-1 and each hub holds
    hub_len random rows, so product column `hubs` has ~29,000 distinct rows:
    more than the multi-pass LDS kernel holds (21,296 keys).  Other columns
    hold their own row and two random rows."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    r, c = [], []
    for k in range(hubs):
        rr = rng.choice(n, size=hub_len, replace=False)
        r.append(rr)
        c.append(np.full(hub_len, k))
    r.append(np.arange(hubs))
    c.append(np.full(hubs, hubs))
    rest = np.arange(hubs + 1, n)
    r += [rest, rng.integers(0, n, rest.size), rng.integers(0, n, rest.size)]
    c += [rest, rest, rest]
    r, c = np.concatenate(r), np.concatenate(c)
    M = sp.csc_matrix((rng.uniform(0.5, 1.0, r.size), (r, c)), shape=(n, n))
    M.sum_duplicates()
    M.sort_indices()
    return oracle.normalize(CSC.from_scipy(M))


def test_overflow_resolves_for_any_estimate(mcl):
    """Estimates far too small (est_scale 1e-9, an untrained MLP) make the
    largest product column overflow every LDS table; it is then sized by its
    exact count and the result is still the oracle's."""
    A = _hub_graph()
    C, flops, nnz = oracle.expand(A, A)
    assert nnz.max() > 21296
    dA = up(mcl, A)
    _, packed = mcl.mlp_init(11)          # untrained network
    for kw in (dict(est_scale=1e-9), dict(estimator=mcl.EST_MLP, mlp_weights=packed),
               dict(estimator=mcl.EST_MLP, mlp_weights=packed, est_scale=1e-9)):
        print("sizing", {k: v for k, v in kw.items() if k != "mlp_weights"}, flush=True)
        G, st = mcl.expand(dA, dA, **kw)
        assert_same_matrix(G.to_host(), C, exact=True)
        _, _, st2 = check_iterate(mcl, A, **kw)
        if kw.get("est_scale") == 1e-9:
            assert st["n_overflow"] > 0 and st2["n_overflow"] > 0


def test_phased_iterate_matches_oracle(mcl):
    """Phases (column ranges with their own temp storage) against the oracle,
    not only against the unphased GPU run."""
    A = oracle.normalize(planted_graph(8000, 250, s_cap=900, seed=25))
    for pb in (3 << 20, 400 << 10):
        _, _, st = check_iterate(mcl, A, phase_bytes=pb)
        assert st["n_phases"] > 1


def test_dense_accumulator_columns_match_oracle(mcl):
    """Components with contiguous vertex ids: product columns whose rows span
    at most 8,192 consecutive rows and that do at least two multiply-adds per
    row of the span go to the dense accumulator (a 9,000-vertex component stays
    on the hash tables).  Two fused iterations, the second from the oracle's
    first iterate (denser columns), and the plain product equal the oracle."""
    U = planted_components([6000, 3000, 1500, 400, 9000, 120], [60, 30, 15, 4, 90, 2], s_cap=600, seed=77)
    A = oracle.normalize(U)
    _, _, st = check_iterate(mcl, A)
    assert st["n_dense"] > 0
    A1, _ = oracle.iterate(A)
    _, _, st1 = check_iterate(mcl, A1)
    assert st1["n_dense"] > 0
    E, _ = mcl.expand(up(mcl, A1), up(mcl, A1))
    ref = oracle.expand(A1, A1)[0]
    e = E.to_host()
    assert np.array_equal(e.colptr, ref.colptr) and np.array_equal(e.rowidx, ref.rowidx)
    assert np.array_equal(e.val, ref.val)
