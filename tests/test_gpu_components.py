"""GPU connected components (the clusters Alg. 1 returns) against the
oracle's components (scipy weak components, smallest vertex id as label), and
whole MCL runs clustered on the GPU against the oracle's MCL."""
import numpy as np
import pytest

import oracle
from mclgen import CSC, config0_graph, planted_components, planted_graph, random_csc, random_symmetric_graph

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


def test_run_mcl_checkpoint_resume_and_log(mcl, tmp_path):
    """An MCL run interrupted after three iterations and resumed from its
    checkpoint ends bit-identical to an uninterrupted run; the per-iteration
    log holds one line per iteration done."""
    import json
    from paper_2002_10083_amd import drivers
    A = oracle.normalize(planted_graph(5000, 200, s_cap=400, seed=41))
    ref, it_ref, lab_ref, nc_ref, conv_ref = drivers.run_mcl(mcl.DeviceCSC.from_host(A), max_iter=100)
    assert conv_ref and it_ref > 3
    ck, log = str(tmp_path / "ck.npz"), str(tmp_path / "log.jsonl")
    _, it1, _, _, conv1 = drivers.run_mcl(mcl.DeviceCSC.from_host(A), max_iter=3, log_path=log,
                                          checkpoint_path=ck, checkpoint_every=2)
    assert it1 == 3 and not conv1
    G, it2, lab, nc, conv = drivers.run_mcl(None, max_iter=100, log_path=log, checkpoint_path=ck, resume=True)
    assert (it2, nc, conv) == (it_ref, nc_ref, conv_ref)
    assert torch.equal(G.colptr, ref.colptr) and torch.equal(G.rowidx, ref.rowidx) and torch.equal(G.val, ref.val)
    assert torch.equal(lab, lab_ref)
    lines = [json.loads(l) for l in open(log)]
    assert [d["iteration"] for d in lines] == list(range(1, it_ref + 1))
    assert lines[-1]["change"] < 1e-9 <= lines[-2]["change"]
    # resuming a finished run does no further iteration
    _, it3, _, _, conv3 = drivers.run_mcl(None, max_iter=100, checkpoint_path=ck, resume=True)
    assert (it3, conv3) == (it_ref, True)
