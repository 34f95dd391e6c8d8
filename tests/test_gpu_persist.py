"""The persistent accumulation (bin_policy bit 28: one launch for the columns
of LDS bins 0-6, waves taking (column, part) items from per-XCD queues in
either bin order, then the finishing launches of every bin) gives the same
bytes as the per-bin launches and matches the oracle: single graphs, expand
mode, forced overflow, dense-accumulator columns and the batched form."""
import numpy as np
import pytest

import oracle
from mclgen import planted_components, planted_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PERSIST = 1 << 28
LIGHT_FIRST = 1 << 29


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def up(m, M):
    return m.DeviceCSC.from_host(M)


def same(X, Y):
    assert torch.equal(X.colptr, Y.colptr)
    assert torch.equal(X.rowidx, Y.rowidx)
    assert torch.equal(X.val, Y.val)


def test_persistent_iterate_and_expand_match_per_bin_launches_and_oracle(mcl):
    A = oracle.normalize(planted_graph(40000, 2000, s_cap=2100, seed=71))
    dA = up(mcl, A)
    ref, c0, st0 = mcl.iterate(dA)
    G, c1, st1 = mcl.iterate(dA, bin_policy=PERSIST)
    assert max(st1["bin_cols"][:7]) > 0 and st1["bin_cols"][6] > 0
    same(G, ref)
    assert c1 == c0
    G2, c2, _ = mcl.iterate(dA, bin_policy=PERSIST | LIGHT_FIRST)  # the other queue order
    same(G2, ref)
    assert c2 == c0
    assert st1["nnz_product"] == st0["nnz_product"] and st1["n_selected"] == st0["n_selected"]
    E0, _ = mcl.expand(dA, dA)
    E1, _ = mcl.expand(dA, dA, bin_policy=PERSIST)
    same(E1, E0)
    R, _, _ = oracle.expand(A, A)
    e = E1.to_host()
    assert np.array_equal(e.colptr, R.colptr) and np.array_equal(e.rowidx, R.rowidx)
    assert np.array_equal(e.val, R.val)


def test_persistent_with_forced_overflow(mcl):
    A = oracle.normalize(planted_graph(20000, 800, s_cap=1500, seed=72))
    dA = up(mcl, A)
    ref, _, _ = mcl.iterate(dA)
    for scale in (0.3, 0.01):
        G, _, st = mcl.iterate(dA, bin_policy=PERSIST, est_scale=scale)
        assert st["n_overflow"] > 0
        same(G, ref)


def test_persistent_batched_with_dense_columns(mcl):
    U = planted_components([6000, 3000, 1500, 400, 9000, 120, 8], [60, 30, 15, 4, 90, 2, 1], s_cap=600, seed=77)
    A = oracle.normalize(U)
    dA = up(mcl, A)
    comp = torch.from_numpy(U.comp_ptr).cuda()
    active = torch.tensor([1, 1, 0, 1, 1, 1, 1], dtype=torch.uint8, device="cuda")
    ref, ch0, st0 = mcl.iterate(dA, comp_ptr=comp, active=active)
    G, ch1, st1 = mcl.iterate(dA, comp_ptr=comp, active=active, bin_policy=PERSIST)
    assert st1["n_dense"] > 0
    same(G, ref)
    assert np.array_equal(ch0, ch1)
    # a second iteration from the oracle's first iterate (denser columns,
    # more of them dense-accumulated); the per-bin launches on the same input
    # match the oracle in test_dense_accumulator_columns_match_oracle
    A1, _ = oracle.iterate(A)
    d1 = up(mcl, A1)
    R1, _, _ = mcl.iterate(d1)
    G1, _, st = mcl.iterate(d1, bin_policy=PERSIST)
    assert st["n_dense"] > 0
    same(G1, R1)
