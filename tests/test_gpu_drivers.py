"""GPU drivers against the oracle: SUMMA-stage partial products merged with
the binary schedule of Alg. 2 (and with one flat merge), and batched MCL to
convergence against the per-component loop."""
import numpy as np
import pytest

import oracle
from mclgen import CSC, planted_components, planted_graph

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def drv():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import drivers, mcl
    return drivers, mcl


def _stage_partials(A, nstages, drivers):
    S = A.to_scipy()
    parts = []
    for k0, k1 in drivers.stage_ranges(A.ncols, nstages):
        Ak = CSC.from_scipy(S[:, k0:k1])
        Bk = CSC.from_scipy(S[k0:k1, :])
        parts.append(oracle.expand(Ak, Bk)[0])
    return parts


@pytest.mark.parametrize("nstages", [8, 5])
def test_summa_merge_matches_oracle(drv, nstages):
    drivers, mcl = drv
    A = oracle.normalize(planted_graph(3000, 120, s_cap=300, seed=41))
    parts = _stage_partials(A, nstages, drivers)
    dA = mcl.DeviceCSC.from_host(A)
    for schedule, ref in (("binary", oracle.binary_merge(parts)[0]), ("flat", oracle.merge(parts))):
        C, info = drivers.summa_merge(dA, nstages, schedule)
        g = C.to_host()
        assert np.array_equal(g.colptr, ref.colptr)
        assert np.array_equal(g.rowidx, ref.rowidx)
        assert np.array_equal(g.val, ref.val)
        assert info["partial_nnz"] == [p.nnz for p in parts]
    # the merged pattern is the pattern of A*A; values agree to rounding
    direct, _, _ = oracle.expand(A, A)
    assert np.array_equal(g.rowidx, direct.rowidx)
    assert np.allclose(g.val, direct.val, rtol=1e-13, atol=0)


def test_summa_stage_blocks(drv):
    drivers, mcl = drv
    A = oracle.normalize(planted_graph(2000, 80, s_cap=200, seed=42))
    S = A.to_scipy()
    dA = mcl.DeviceCSC.from_host(A)
    for k0, k1 in drivers.stage_ranges(A.ncols, 3):
        for got, ref in ((drivers.column_block(dA, k0, k1), S[:, k0:k1]),
                         (drivers.row_block(dA, k0, k1), S[k0:k1, :])):
            r = CSC.from_scipy(ref)
            g = got.to_host()
            assert (g.nrows, g.ncols) == (r.nrows, r.ncols)
            assert np.array_equal(g.colptr, r.colptr)
            assert np.array_equal(g.rowidx, r.rowidx)
            assert np.array_equal(g.val, r.val)


def test_batched_mcl_equals_component_loop(drv):
    drivers, mcl = drv
    U = planted_components([300, 40, 1200, 8, 900, 3], [12, 2, 50, 1, 36, 1], s_cap=300, seed=43)
    A = oracle.normalize(U)
    comp = torch.from_numpy(U.comp_ptr).cuda()
    Af, iters, info = drivers.batched_mcl(mcl.DeviceCSC.from_host(A), comp)
    assert info["calls"] == iters.max()
    assert info["not_converged"] == 0 and info["converged"].all()
    lab, ncomp = mcl.components(Af)
    lab = lab.cpu().numpy().astype(np.int64)
    nclusters = 0
    for c in range(len(U.comp_ptr) - 1):
        c0, c1 = int(U.comp_ptr[c]), int(U.comp_ptr[c + 1])
        blk_h = drivers.component_block(A, c0, c1)
        Bf, it, conv = drivers.component_mcl(mcl.DeviceCSC.from_host(blk_h))
        assert conv
        assert it == iters[c], c
        assert drivers.same_block(Af, c0, c1, Bf), c
        # the batched result clusters every component as the oracle's MCL
        # of that component alone does (labels offset by the block start)
        _, it_o, lab_o = oracle.mcl(blk_h, normalized=True)
        assert abs(it_o - it) <= 1, c
        assert np.array_equal(lab[c0:c1], lab_o + c0), c
        nclusters += len(np.unique(lab_o))
    assert ncomp == nclusters


def test_summa_merge_large_columns(drv):
    # merged columns of ~10,800 rows: beyond the largest LDS table (HBM tables)
    drivers, mcl = drv
    A = oracle.normalize(planted_graph(12000, 2, s_cap=11000, p_in=0.02, x=0.0, seed=64))
    parts = _stage_partials(A, 4, drivers)
    ref, _ = oracle.binary_merge(parts)
    C, info = drivers.summa_merge(mcl.DeviceCSC.from_host(A), 4, "binary")
    g = C.to_host()
    assert np.array_equal(g.colptr, ref.colptr)
    assert np.array_equal(g.rowidx, ref.rowidx)
    assert np.array_equal(g.val, ref.val)


_STRIPES = {}


def _stripe_case():
    """Stripe blocks of a 480,000-vertex planted graph (8 x 8 grid, position
    (0, 1)) and the oracle's 8 stage products (computed once)."""
    if not _STRIPES:
        from mclgen.planted import stripe_blocks
        R, Cb = stripe_blocks(N=480_000, grid=8, row_stripe=0, col_stripe=1, workers=4)
        _STRIPES["case"] = (R, Cb, [oracle.expand(R[k], Cb[k])[0] for k in range(8)])
    return _STRIPES["case"]


@pytest.mark.parametrize("schedule", ["binary", "flat"])
def test_stripe_blocks_overlapped_merge_matches_oracle(drv, schedule):
    """One process's SUMMA share of a 2D-distributed planted graph (8 x 8
    grid, position (0, 1), scaled down to 480,000 vertices): the overlapped
    driver (merges on a second stream) equals the one-stream driver bit for
    bit, and both equal the oracle's stage products merged by its heap merge
    with the same schedule."""
    drivers, mcl = drv
    R, Cb, parts = _stripe_case()
    dR = [mcl.DeviceCSC.from_host(x) for x in R]
    dC = [mcl.DeviceCSC.from_host(x) for x in Cb]
    ops = lambda i: (dR[i], dC[i])
    C1, i1 = drivers.summa_stages(ops, 8, schedule)
    C2, i2 = drivers.summa_stages_overlapped(ops, 8, schedule)
    assert i2["merges"] == i1["merges"] == ([2, 3, 2, 4] if schedule == "binary" else [8])
    assert torch.equal(C1.colptr, C2.colptr) and torch.equal(C1.rowidx, C2.rowidx)
    assert torch.equal(C1.val, C2.val)
    assert i2["peak_list_bytes"] >= max(drivers.csc_bytes(C1), 1)
    ref = oracle.binary_merge(parts)[0] if schedule == "binary" else oracle.merge(parts)
    g = C2.to_host()
    assert np.array_equal(g.colptr, ref.colptr) and np.array_equal(g.rowidx, ref.rowidx)
    assert np.array_equal(g.val, ref.val)
