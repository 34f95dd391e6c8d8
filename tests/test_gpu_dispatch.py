"""The CPU/GPU dispatch by flops (mcl_expand_dispatch, Section 3) on the GPU
leg: host matrices copied to the device, expanded there and copied back, bit
for bit the same as the CPU hash SpGEMM and the oracle."""
import numpy as np
import pytest

import oracle
from mclgen import planted_graph, random_csc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def _same(C, R):
    assert np.array_equal(C.colptr, R.colptr)
    assert np.array_equal(C.rowidx, R.rowidx)
    assert np.array_equal(C.val.view(np.uint64), R.val.view(np.uint64))


def test_dispatch_gpu_leg_matches_host_spgemm_and_oracle(mcl):
    A = oracle.normalize(planted_graph(12000, 480, s_cap=900, seed=21))
    R, flops, _ = oracle.expand(A, A)
    C, st, where = mcl.expand_dispatch(A, A, gpu_min_flops=1)
    assert where == "gpu"
    assert st["flops"] == int(np.asarray(flops).sum())
    _same(C, R)
    H, _ = mcl.expand_host(A, A)
    _same(H, R)


def test_dispatch_default_threshold_sends_large_products_to_the_gpu(mcl):
    A = oracle.normalize(planted_graph(30000, 1200, s_cap=1500, seed=22))
    _, flops, _ = oracle.expand(A, A)
    assert int(np.asarray(flops).sum()) >= mcl.DISPATCH_GPU_MIN_FLOPS
    C, st, where = mcl.expand_dispatch(A, A)
    assert where == "gpu"
    H, _ = mcl.expand_host(A, A)
    _same(C, H)


def test_dispatch_rectangular_and_empty_columns(mcl):
    A = random_csc(3000, 2000, 9, seed=23, skew=1.0)
    B = random_csc(2000, 1700, 6, seed=24, skew=1.0, empty_frac=0.1)
    R, _, _ = oracle.expand(A, B)
    for cut in (1, 1 << 40):
        C, _, where = mcl.expand_dispatch(A, B, gpu_min_flops=cut)
        assert where == ("gpu" if cut == 1 else "cpu")
        _same(C, R)
