"""What the trained network gains over the method without it (the learned
estimator replacing Cohen's, Section 5): an MLP trained with the library's
kernels on rows logged from other seeds sizes the tables of a held-out
graph with fewer overflowed and fewer HBM-table columns than Cohen's
estimator, and the pruned result is bit-identical."""
import pytest
import torch

from mclgen import config1_graph

pytestmark = pytest.mark.gpu

N = 200_000


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_10083_amd import mcl as m
    return m


def _graph(mcl, seed):
    A = mcl.DeviceCSC.from_host(config1_graph(seed=seed, n=N, n_clusters=N // 20))
    mcl.normalize_(A)
    return A


def test_trained_mlp_sizes_better_than_cohen(mcl):
    from paper_2002_10083_amd import learned
    base = dict(cohen_keys=12)
    Xs, ys = [], []
    for sd in (3001, 3002, 3003):
        X, y = learned.collect(_graph(mcl, sd), iterations=3, params=mcl.default_params(**base))
        Xs.append(X)
        ys.append(y)
    state, packed, losses = learned.train(torch.cat(Xs), torch.cat(ys), epochs=24, decay=0.85)
    assert losses[-1] < 0.25 * losses[0]
    mlp_kw = dict(estimator=mcl.EST_MLP, mlp_weights=packed)
    q = learned.residual_quantiles(_graph(mcl, 3004), mlp_kw, iterations=1, params=mcl.default_params(**base))
    scale = learned.scale_for_quantile(q, 0.75)
    A = _graph(mcl, 3005)
    Gc, _, sc = mcl.iterate(A, mcl.default_params(**base, estimator=mcl.EST_COHEN))
    Gm, _, sm = mcl.iterate(A, mcl.default_params(**base, **mlp_kw, est_scale=scale))
    print("cohen overflow %d global %d total %.2f ms | mlp (scale %.3f) overflow %d global %d total %.2f ms"
          % (sc["n_overflow"], sc["n_global"], sc["t_total_ms"], scale, sm["n_overflow"], sm["n_global"],
             sm["t_total_ms"]))
    assert torch.equal(Gc.colptr, Gm.colptr)
    assert torch.equal(Gc.rowidx, Gm.rowidx)
    assert torch.equal(Gc.val, Gm.val)
    assert sm["n_overflow"] < sc["n_overflow"]
    assert sm["n_global"] <= sc["n_global"]
