"""mcl_components_noalloc (the entry point for callers that cannot allocate
device memory) against mcl_components, which takes its scratch from the
allocator: identical labels and component counts, on consecutive calls that
share the library's one scratch array, the second on a smaller graph; the
oracle's components pin both."""
import numpy as np
import pytest

import oracle
from mclgen import CSC, random_csc, random_symmetric_graph

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def _both(mcl, M):
    D = mcl.DeviceCSC.from_host(M)
    ref_lab, ref_nc = mcl.components(D)
    lab, nc = mcl.components_noalloc(D)
    return (lab.cpu().numpy().astype(np.int64), nc,
            ref_lab.cpu().numpy().astype(np.int64), ref_nc)


def test_noalloc_matches_allocating_entry_on_consecutive_calls(mcl):
    big = random_csc(300_000, 300_000, 0.9, seed=11)      # many components and singletons
    small = random_symmetric_graph(2_000, 0.002, seed=12)
    for name, M in (("big", big), ("small", small), ("big-again", big)):
        print("case", name, M.ncols, flush=True)
        lab, nc, ref_lab, ref_nc = _both(mcl, M)
        assert np.array_equal(lab, ref_lab), name
        assert nc == ref_nc, name
        assert np.array_equal(lab, oracle.clusters(M)), name


def test_noalloc_without_sync_and_into_caller_labels(mcl):
    M1 = random_csc(50_000, 50_000, 1.1, seed=21)
    M2 = random_csc(7_000, 7_000, 0.7, seed=22)
    for M in (M1, M2):
        D = mcl.DeviceCSC.from_host(M)
        out = torch.full((M.ncols,), -7, dtype=torch.int32, device="cuda")
        lab, nc = mcl.components_noalloc(D, labels=out, sync=False)
        assert nc is None and lab.data_ptr() == out.data_ptr()
        torch.cuda.synchronize()
        ref_lab, _ = mcl.components(D)
        assert torch.equal(out, ref_lab)


def _sparse_random_pattern(n, m, seed):
    """n x n pattern with about m random entries (duplicates merged)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, m)
    c = rng.integers(0, n, m)
    S = sp.csc_matrix((np.ones(m), (r, c)), shape=(n, n))
    S.sum_duplicates()
    S.sort_indices()
    return CSC.from_scipy(S)


def test_noalloc_at_the_size_limit_and_beyond(mcl):
    n = mcl.NOALLOC_MAX_VERTICES
    M = _sparse_random_pattern(n, n // 2, seed=31)
    print("case limit", n, flush=True)
    lab, nc, ref_lab, ref_nc = _both(mcl, M)
    assert np.array_equal(lab, ref_lab) and nc == ref_nc
    # one vertex more is refused before any kernel runs
    n1 = n + 1
    big = CSC(n1, n1, np.zeros(n1 + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(mcl.MclError, match="scratch limit"):
        mcl.components_noalloc(mcl.DeviceCSC.from_host(big))
    # the scratch is still good after the refused call
    small = random_symmetric_graph(500, 0.01, seed=32)
    lab, nc, ref_lab, ref_nc = _both(mcl, small)
    assert np.array_equal(lab, ref_lab) and nc == ref_nc


def test_noalloc_empty_and_non_square(mcl):
    E = CSC(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    lab, nc = mcl.components_noalloc(mcl.DeviceCSC.from_host(E))
    assert nc == 0 and lab.numel() == 0
    R = random_csc(30, 20, 2.0, seed=41)
    with pytest.raises(mcl.MclError, match="square"):
        mcl.components_noalloc(mcl.DeviceCSC.from_host(R))
