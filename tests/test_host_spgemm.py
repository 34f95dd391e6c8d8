"""The library's multithreaded CPU hash SpGEMM (mcl_expand_host, Section 6
"Faster SpGEMM on CPU") and the CPU leg of the flops dispatch
(mcl_expand_dispatch, Section 3): bit-exact against the oracle's expansion,
independent of the thread count, and the structure checks of the host
entry points.  Runs on the CPU (no GPU call is made)."""
import os

import numpy as np
import pytest

import oracle
from mclgen import CSC, planted_graph, random_csc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2002_10083_amd", "libmcl.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmcl.so not built")


def _same(C, R):
    assert C.nrows == R.nrows and C.ncols == R.ncols
    assert np.array_equal(C.colptr, R.colptr)
    assert np.array_equal(C.rowidx, R.rowidx)
    # bit-exact: the same ascending-k order of rounded products
    assert np.array_equal(C.val.view(np.uint64), R.val.view(np.uint64))


CASES = [
    ("rectangular", lambda: (random_csc(300, 200, 7, seed=1, skew=0.8),
                             random_csc(200, 150, 5, seed=2, skew=0.8, empty_frac=0.1))),
    ("planted", lambda: (lambda A: (A, A))(oracle.normalize(planted_graph(6000, 240, s_cap=500, seed=3)))),
    ("skewed", lambda: (random_csc(5000, 4000, 20, seed=4, skew=1.6),
                        random_csc(4000, 3000, 12, seed=5, skew=1.6, empty_frac=0.2))),
    ("one_dense_row", lambda: (lambda A, B: (A, B))(
        CSC(64, 1, np.array([0, 64], np.int64), np.arange(64, dtype=np.int32), np.linspace(0.1, 1, 64)),
        CSC(1, 50, np.arange(51, dtype=np.int64), np.zeros(50, np.int32), np.linspace(1, 2, 50)))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_expand_host_is_bit_exact_vs_oracle(name, make):
    from paper_2002_10083_amd import mcl
    A, B = make()
    R, flops, _ = oracle.expand(A, B)
    C, st = mcl.expand_host(A, B, nthreads=4)
    _same(C, R)
    assert st["flops"] == int(np.asarray(flops).sum())
    assert st["nnz_product"] == R.nnz


def test_expand_host_thread_count_does_not_change_bits():
    from paper_2002_10083_amd import mcl
    A = oracle.normalize(planted_graph(4000, 150, s_cap=400, seed=9))
    C1, _ = mcl.expand_host(A, A, nthreads=1)
    for t in (2, 7, 0):
        Ct, st = mcl.expand_host(A, A, nthreads=t)
        _same(Ct, C1)


def test_expand_host_empty_shapes():
    from paper_2002_10083_amd import mcl
    z = CSC(5, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    e = CSC(0, 5, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    C, st = mcl.expand_host(e, z)  # 0x5 times 5x0
    assert (C.nrows, C.ncols, C.nnz) == (0, 0, 0)
    B = CSC(5, 3, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))  # all columns empty
    A = random_csc(7, 5, 3, seed=1)
    C, st = mcl.expand_host(A, B)
    assert C.nnz == 0 and np.array_equal(C.colptr, np.zeros(4, np.int64)) and st["flops"] == 0


def test_expand_host_rejects_malformed_input():
    from paper_2002_10083_amd import mcl
    A = random_csc(20, 20, 4, seed=2)
    bad = CSC(A.nrows, A.ncols, A.colptr.copy(), A.rowidx.copy(), A.val.copy())
    bad.rowidx[3] = 20  # row out of range
    with pytest.raises(mcl.MclError) as e:
        mcl.expand_host(bad, A)
    assert e.value.code == mcl.MCL_EINVAL and "out of range" in str(e.value)
    dec = CSC(A.nrows, A.ncols, A.colptr.copy(), A.rowidx.copy(), A.val.copy())
    dec.colptr[5], dec.colptr[6] = dec.colptr[6], dec.colptr[5] - 1
    with pytest.raises(mcl.MclError):
        mcl.expand_host(dec, A)
    with pytest.raises(mcl.MclError) as e:
        mcl.expand_host(A, random_csc(21, 4, 2, seed=3))  # A.ncols != B.nrows
    assert e.value.code == mcl.MCL_EINVAL


def test_dispatch_keeps_small_products_on_the_cpu():
    from paper_2002_10083_amd import mcl
    A = oracle.normalize(planted_graph(1000, 50, s_cap=80, seed=11))
    R, flops, _ = oracle.expand(A, A)
    total = int(np.asarray(flops).sum())
    assert total < mcl.DISPATCH_GPU_MIN_FLOPS
    C, st, where = mcl.expand_dispatch(A, A)  # default threshold
    assert where == "cpu"
    _same(C, R)
    C, st, where = mcl.expand_dispatch(A, A, gpu_min_flops=total + 1, nthreads=3)
    assert where == "cpu" and st["flops"] == total
    _same(C, R)
