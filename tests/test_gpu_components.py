"""GPU connected components (the clusters Alg. 1 returns) against the
oracle's components (scipy weak components, smallest vertex id as label), and
whole MCL runs clustered on the GPU against the oracle's MCL."""
import numpy as np
import pytest

import oracle
from mclgen import CSC, config0_graph, planted_components, random_csc, random_symmetric_graph

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def _path_graph(n, seed):
    """A path through all n vertices in random order (one component whose
    union-find trees can grow deep), with one-directional entries only."""
    order = np.random.default_rng(seed).permutation(n)
    rows = order[1:].astype(np.int64)
    cols = order[:-1].astype(np.int64)
    import scipy.sparse as sp
    M = sp.csc_matrix((np.ones(n - 1), (rows, cols)), shape=(n, n))
    M.sort_indices()
    return CSC.from_scipy(M)


def _labels(mcl, M):
    lab, nc = mcl.components(mcl.DeviceCSC.from_host(M))
    return lab.cpu().numpy().astype(np.int64), nc


@pytest.mark.parametrize("case", ["sym", "directed", "sparse", "path", "isolated", "empty", "one"])
def test_components_match_oracle(mcl, case):
    print("case", case, flush=True)
    if case == "sym":
        M = random_symmetric_graph(3000, 0.0008, seed=1)
    elif case == "directed":       # pattern not symmetric: weak connectivity
        M = random_csc(5000, 5000, 1.2, seed=2)
    elif case == "sparse":         # many small components and singletons
        M = random_csc(20000, 20000, 0.6, seed=3)
    elif case == "path":
        M = _path_graph(100000, seed=4)
    elif case == "isolated":       # only self-loops: every vertex alone
        n = 777
        M = CSC(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    elif case == "empty":          # no entries at all
        n = 64
        M = CSC(n, n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    else:
        M = CSC(1, 1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([1.0]))
    ref = oracle.clusters(M)
    lab, nc = _labels(mcl, M)
    assert np.array_equal(lab, ref)
    assert nc == len(np.unique(ref))


def test_components_zero_vertices(mcl):
    M = CSC(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    lab, nc = mcl.components(mcl.DeviceCSC.from_host(M))
    assert lab.numel() == 0 and nc == 0


def test_components_reject_rectangular(mcl):
    M = random_csc(30, 20, 2, seed=5)
    with pytest.raises(mcl.MclError) as e:
        mcl.components(mcl.DeviceCSC.from_host(M))
    assert e.value.code == mcl.MCL_EINVAL


def test_mcl_clusters_on_gpu_match_oracle(mcl):
    """The 10,000-vertex planted graph run to convergence on the GPU and
    clustered on the GPU: the oracle's clusters and iteration count (+-1)."""
    from paper_2002_10083_amd import drivers
    W = config0_graph()
    Ao, it_o, lab_o = oracle.mcl(W)
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)
    Af, it, lab, nc, conv = drivers.run_mcl(A)
    assert conv
    lab = lab.cpu().numpy().astype(np.int64)
    assert np.array_equal(lab, oracle.clusters(Af.to_host()))   # same labelling of the same pattern
    assert np.array_equal(lab, lab_o)                            # the oracle's own run
    assert nc == len(np.unique(lab_o))
    assert abs(it - it_o) <= 1
