"""GPU kernels of the learned estimator against the MLP oracle: BF16 forward
(bit-exact), gradient and Adam step, training progress, the 12 features, and
byte-identical iterations when the MLP sizes the tables."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from mclgen import planted_graph

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mcl():
    assert torch.cuda.is_available()
    from paper_2002_10083_amd import mcl as m
    return m


def _params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(omlp.NPARAM, np.float32)
    p[omlp.OFF_W1:omlp.OFF_B1] = rng.uniform(-1, 1, 768) * np.sqrt(0.5)
    p[omlp.OFF_B1:omlp.OFF_W2] = rng.uniform(-0.1, 0.1, 64)
    p[omlp.OFF_W2:omlp.OFF_B2] = rng.uniform(-1, 1, 4096) * np.sqrt(6 / 64)
    p[omlp.OFF_B2:omlp.OFF_W3] = rng.uniform(-0.1, 0.1, 64)
    p[omlp.OFF_W3:omlp.OFF_B3] = rng.uniform(-1, 1, 64) * np.sqrt(6 / 64)
    p[omlp.OFF_B3] = 0.5
    return p


def _state_with(mcl, p):
    state, packed = mcl.mlp_init(0)
    state.zero_()
    state[:omlp.NPARAM] = torch.from_numpy(p).cuda()
    # a zero-learning-rate step packs the BF16 weights without moving them
    X = torch.zeros(256, 12, device="cuda")
    mcl.mlp_train_step(state, packed, X, torch.zeros(256, device="cuda"), lr=0.0)
    assert torch.equal(state[:omlp.NPARAM].cpu(), torch.from_numpy(p))
    state[5120:] = 0.0          # fresh Adam moments and step counter
    return state, packed


def test_forward_bit_exact(mcl):
    p = _params(1)
    _, packed = _state_with(mcl, p)
    X = np.random.default_rng(2).uniform(0, 8, (5000, 12)).astype(np.float32)
    got = mcl.mlp_forward(packed, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = omlp.forward_f32(p, X)
    assert np.array_equal(got, ref)


def test_gradient_and_adam_step(mcl):
    p = _params(3)
    state, packed = _state_with(mcl, p)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 6, (3000, 12)).astype(np.float32)
    y = rng.uniform(0, 8, 3000).astype(np.float32)
    s0 = state.clone()
    lr = 1e-3
    loss, g = mcl.mlp_train_step(state, packed, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                                 lr=lr, want_grad=True)
    ref_loss, ref_g, _ = omlp.forward_backward(p, X, y, casts=True)
    g = g[:omlp.NPARAM].cpu().numpy().astype(np.float64)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    scale = np.abs(ref_g).max()
    assert np.abs(g - ref_g).max() <= 2e-4 * scale
    # the update is one Adam step from zero moments
    q, _, _ = omlp.adam(p.astype(np.float64), 0, 0, g, 1, lr)
    new = state[:omlp.NPARAM].cpu().numpy()
    assert np.allclose(new, q, rtol=1e-5, atol=1e-7)
    assert float(state[3 * 5120].cpu()) == 1.0
    del s0


def test_training_reduces_loss(mcl):
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 5, (20000, 12)).astype(np.float32)
    y = (0.8 * X[:, 1] + 0.3 * X[:, 2] - 0.1 * X[:, 5] + 1.0).astype(np.float32)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    state, packed = mcl.mlp_init(7)
    first = mcl.mlp_train_step(state, packed, Xd, yd, lr=3e-3)
    for _ in range(300):
        last = mcl.mlp_train_step(state, packed, Xd, yd, lr=3e-3)
    assert last < 0.02 * first


def test_features_match_definitions(mcl):
    A = oracle.normalize(planted_graph(3000, 120, s_cap=300, seed=8))
    dA = mcl.DeviceCSC.from_host(A)
    _, F = mcl.estimate(dA, dA, features=True, iteration=2)
    ref = omlp.features(A.colptr, A.rowidx, A.colptr, A.rowidx, A.val, 2)
    got = F.cpu().numpy().astype(np.float64)
    assert np.allclose(got, ref, rtol=2e-5, atol=1e-5)


def test_iterate_with_mlp_sizing_is_identical(mcl):
    A = oracle.normalize(planted_graph(8000, 250, s_cap=900, seed=9))
    dA = mcl.DeviceCSC.from_host(A)
    state, packed = mcl.mlp_init(11)   # untrained: poor sizing, many overflows
    ref, c0, _ = mcl.iterate(dA, estimator=mcl.EST_COHEN)
    X, c1, st = mcl.iterate(dA, estimator=mcl.EST_MLP, mlp_weights=packed)
    assert torch.equal(X.rowidx, ref.rowidx) and torch.equal(X.val, ref.val) and c0 == c1
