"""Pins of the learned-estimator oracle: BF16 rounding on hand-worked
values, the FP32 forward against the FP64 forward, and the analytic
gradient against central finite differences (casts off)."""
import numpy as np

from oracle import mlp


def test_bf16_round_hand_values():
    def f(bits):
        return np.array([bits], np.uint32).view(np.float32)
    cases = [
        (0x3F800000, 0x3F800000),   # 1.0 exact
        (0x3F808000, 0x3F800000),   # 1 + 2^-8: tie -> even (1.0)
        (0x3F818000, 0x3F820000),   # 1 + 2^-7 + 2^-8: tie -> even (1 + 2^-6)
        (0x3F808001, 0x3F810000),   # just above the tie -> up
        (0x3F807FFF, 0x3F800000),   # just below the tie -> down
        (0xBF808001, 0xBF810000),   # negative, away from zero
        (0x40490FDB, 0x40490000),   # pi -> 3.140625
        (0x00000000, 0x00000000),
    ]
    for src, want in cases:
        got = mlp.bf16_round(f(src)).view(np.uint32)[0]
        assert got == want, (hex(src), hex(got), hex(want))


def _params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_W1:mlp.OFF_B1] = rng.uniform(-1, 1, mlp.NH * mlp.NIN) * np.sqrt(6 / 12)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.uniform(-0.1, 0.1, mlp.NH)
    p[mlp.OFF_W2:mlp.OFF_B2] = rng.uniform(-1, 1, mlp.NH * mlp.NH) * np.sqrt(6 / 64)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.uniform(-0.1, 0.1, mlp.NH)
    p[mlp.OFF_W3:mlp.OFF_B3] = rng.uniform(-1, 1, mlp.NH) * np.sqrt(6 / 64)
    p[mlp.OFF_B3] = 0.3
    return p


def test_forward_f32_close_to_f64_with_casts():
    p = _params(1).astype(np.float32)
    X = np.random.default_rng(2).uniform(0, 5, (300, 12)).astype(np.float32)
    y = np.zeros(300)
    _, _, out64 = mlp.forward_backward(p, X, y, casts=True)
    out32 = mlp.forward_f32(p, X)
    # same casts, FP32 vs FP64 accumulation: BF16 roundings of hidden
    # activations may flip on a few rows, everything else agrees closely
    rel = np.abs(out32 - out64) / np.maximum(np.abs(out64), 1e-3)
    assert np.median(rel) < 1e-6
    assert (rel < 1e-4).mean() > 0.9


def test_gradient_matches_finite_differences():
    p = _params(3)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 3, (64, 12))
    y = rng.uniform(0, 6, 64)
    loss, g, _ = mlp.forward_backward(p, X, y, casts=False)
    idx = np.concatenate([rng.choice(mlp.NPARAM - 1, 60, replace=False), [mlp.OFF_B3]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.forward_backward(pp, X, y, casts=False)[0]
              - mlp.forward_backward(pm, X, y, casts=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_moves_by_lr():
    p = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    q, m, v = mlp.adam(p, np.zeros(4), np.zeros(4), g, 1, 0.01)
    # bias-corrected first step is lr * sign(g) (up to eps)
    assert np.allclose(q[:3], -0.01 * np.sign(g[:3]), rtol=1e-6)
    assert q[3] == 0.0


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 3, (512, 12))
    y = 0.7 * X[:, 0] + np.log1p(X[:, 1] * X[:, 2]) + 0.2
    p = _params(6)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.forward_backward(p, X, y)[0]
    for t in range(1, 301):
        loss, g, _ = mlp.forward_backward(p, X, y)
        p, m, v = mlp.adam(p, m, v, g, t, 3e-3)
    assert loss < 0.05 * l0


def test_adam_second_step_closed_form():
    """Adam's bias-corrected moments after two steps: m2 = 0.09 g1 + 0.1 g2,
    v2 = 0.000999 g1^2 + 0.001 g2^2, divided by 1 - 0.9^2 = 0.19 and
    1 - 0.999^2 = 0.001999.  Constant gradients move every step by lr;
    g = (1, -1) gives m_hat = -1/19 and v_hat = 1 at step 2."""
    lr, eps = 0.01, 1e-8
    p0 = np.zeros(2)
    m0 = np.zeros(2)
    v0 = np.zeros(2)
    g1 = np.array([1.0, 1.0])
    g2 = np.array([1.0, -1.0])
    p1, m1, v1 = mlp.adam(p0, m0, v0, g1, 1, lr)
    p2, m2, v2 = mlp.adam(p1, m1, v1, g2, 2, lr)
    assert np.allclose(m2, [0.19, -0.01], rtol=1e-14)
    assert np.allclose(v2, [0.001999, 0.001999], rtol=1e-14)
    step1 = lr / (1.0 + eps)
    want = np.array([-step1 - step1, -step1 + (lr / 19.0) / (1.0 + eps)])
    assert np.allclose(p2, want, rtol=1e-12, atol=0)


def test_features_hand_worked():
    """The 12 inputs of the learned estimator on a 3-column example worked by
    hand.  A (5 x 4): column 0 = rows {0, 2}, column 1 = rows {1, 3, 4},
    column 2 empty, column 3 = row {4}.  B (4 x 3): column 0 references
    k = 0, 1 with b = 0.5, 0.25; column 1 references only the empty k = 2
    with b = 1; column 2 references k = 0, 1, 3 with b = 0.125, 0.5, 0.25."""
    Acp = np.array([0, 2, 5, 5, 6])
    Ari = np.array([0, 2, 1, 3, 4, 4])
    Bcp = np.array([0, 2, 3, 6])
    Bri = np.array([0, 1, 2, 0, 1, 3])
    Bv = np.array([0.5, 0.25, 1.0, 0.125, 0.5, 0.25])
    F = mlp.features(Acp, Ari, Bcp, Bri, Bv, 3, prev_nnz=np.array([7, 0, 11]))
    L = np.log1p
    want = np.array([
        # nnz(B_j) flops  max   mean    min  it span  bmax  sum b^2   std of nnz(A_k)  prev   sum b*nnz(A_k)
        [L(2), L(5), L(3), L(2.5), L(2), 3, L(5), 0.5, 0.3125, L(0.5), L(7), L(1.75)],
        [L(1), L(0), L(0), L(0), L(0), 3, L(0), 1.0, 1.0, L(0), L(0), L(0)],
        [L(3), L(6), L(3), L(2), L(1), 3, L(5), 0.5, 0.328125, L(np.sqrt(2.0 / 3.0)), L(11), L(2.0)],
    ])
    assert np.allclose(F, want, rtol=1e-15, atol=0), F - want
    # without a previous iteration the tenth input is 0
    assert np.all(mlp.features(Acp, Ari, Bcp, Bri, Bv, 0)[:, 10] == 0.0)
