"""Degenerate shapes through the C ABI: zero columns, one vertex, empty
columns, isolated vertices, a single merge part, all components frozen."""
import numpy as np
import pytest

import oracle
from mclgen import CSC, planted_components, random_csc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def _csc(n, cols):
    colptr = np.zeros(n + 1, np.int64)
    rows, vals = [], []
    for j, c in enumerate(cols):
        rows += [r for r, _ in c]
        vals += [v for _, v in c]
        colptr[j + 1] = len(rows)
    return CSC(n, n, colptr, np.array(rows, np.int32), np.array(vals, np.float64))


def test_zero_columns(mcl):
    A = random_csc(5, 0, 1, seed=1)
    B = random_csc(0, 4, 1, seed=2)
    G, st = mcl.expand(mcl.DeviceCSC.from_host(A), mcl.DeviceCSC.from_host(B))
    g = G.to_host()
    assert g.nrows == 5 and g.ncols == 4 and g.nnz == 0
    assert st["flops"] == 0


def test_single_vertex(mcl):
    A = _csc(1, [[(0, 1.0)]])
    G, change, st = mcl.iterate(mcl.DeviceCSC.from_host(A))
    g = G.to_host()
    assert g.nnz == 1 and g.val[0] == 1.0 and change == 0.0


def test_empty_and_isolated_columns(mcl):
    # column 1 is empty, vertex 3 only has its self-loop
    A = oracle.normalize(_csc(4, [[(0, 1.0), (2, 0.5)], [], [(0, 0.5), (2, 1.0)], [(3, 1.0)]]))
    C, flops, nnz = oracle.expand(A, A)
    G, st = mcl.expand(mcl.DeviceCSC.from_host(A), mcl.DeviceCSC.from_host(A))
    g = G.to_host()
    assert np.array_equal(g.colptr, C.colptr) and np.array_equal(g.rowidx, C.rowidx)
    assert np.array_equal(g.val, C.val)
    An, info = oracle.iterate(A)
    X, change, _ = mcl.iterate(mcl.DeviceCSC.from_host(A))
    x = X.to_host()
    assert np.array_equal(x.colptr, An.colptr) and np.array_equal(x.rowidx, An.rowidx)
    assert np.allclose(x.val, An.val, rtol=1e-12, atol=0)


def test_single_part_merge_is_a_copy(mcl):
    P = random_csc(300, 200, 5, seed=3, empty_frac=0.2)
    G, _ = mcl.merge_partials([mcl.DeviceCSC.from_host(P)])
    g = G.to_host()
    assert np.array_equal(g.colptr, P.colptr) and np.array_equal(g.rowidx, P.rowidx)
    assert np.array_equal(g.val, P.val)


def test_all_components_frozen_is_a_copy(mcl):
    U = planted_components([50, 8, 120], [2, 1, 4], s_cap=60, seed=4)
    A = oracle.normalize(U)
    dA = mcl.DeviceCSC.from_host(A)
    comp = torch.from_numpy(U.comp_ptr).cuda()
    active = torch.zeros(3, dtype=torch.uint8, device="cuda")
    X, change, st = mcl.iterate(dA, comp_ptr=comp, active=active)
    assert torch.equal(X.colptr, dA.colptr) and torch.equal(X.rowidx, dA.rowidx)
    assert torch.equal(X.val, dA.val)
    assert np.all(change == 0.0)
