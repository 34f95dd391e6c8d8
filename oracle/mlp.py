"""Oracle of the learned output-size estimator -- TEST INFRASTRUCTURE.

A 12 -> 64 -> 64 -> 1 ReLU multilayer perceptron predicting log(1 + nnz) of
a product column.  Parameter vector layout (5057 values):
W1[64][12], b1[64], W2[64][64], b2[64], W3[64], b3.

BF16 handling (weights and layer inputs rounded to BF16, round to nearest,
ties to even) is implemented here by choosing between the two neighbouring
BF16 values, a route independent of the kernels' bit arithmetic.  With
casts, every product of two BF16 numbers is exact in FP32, so the forward
pass in FP32 with the bias first and the inputs in index order reproduces
the kernels' accumulation exactly.  The FP64 path (casts off) is the
reference for the analytic gradient, pinned by finite differences.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 12, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + NH * NIN
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest BF16 value (ties to even), as float32.

    The two candidates are the BF16 values just below and just above |x|
    (x with its low 16 bits cleared, and the next BF16 magnitude); the
    nearer one wins, a tie goes to the one with an even last mantissa bit."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32)
    lo_bits = u & np.uint32(0xFFFF0000)
    hi_bits = lo_bits + np.uint32(0x10000)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = hi_bits.view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo = np.abs(xd - lo)
    dhi = np.abs(hi - xd)
    lo_even = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & lo_even)
    out = np.where(pick_lo, lo, hi).astype(np.float32)
    return np.where(np.isfinite(x), out, x)


def unpack(p):
    p = np.asarray(p)
    W1 = p[OFF_W1:OFF_B1].reshape(NH, NIN)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(NH, NH)
    b2 = p[OFF_B2:OFF_W3]
    W3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def forward_f32(params, X):
    """Forward with BF16 casts and FP32 sequential accumulation (bias, then
    inputs in index order) -- the kernels' arithmetic.  X: (rows, 12) float32."""
    wb = bf16_round(np.asarray(params, np.float32))
    W1, b1, W2, b2, W3, b3 = unpack(wb)
    x = bf16_round(np.asarray(X, np.float32))
    rows = x.shape[0]
    acc = np.broadcast_to(b1, (rows, NH)).astype(np.float32).copy()
    for i in range(NIN):
        acc = (acc + (W1[:, i][None, :] * x[:, i:i + 1]).astype(np.float32)).astype(np.float32)
    h1 = bf16_round(np.maximum(acc, np.float32(0)))
    acc = np.broadcast_to(b2, (rows, NH)).astype(np.float32).copy()
    for k in range(NH):
        acc = (acc + (W2[:, k][None, :] * h1[:, k:k + 1]).astype(np.float32)).astype(np.float32)
    h2 = bf16_round(np.maximum(acc, np.float32(0)))
    out = np.full(rows, b3, np.float32)
    for k in range(NH):
        out = (out + (W3[k] * h2[:, k]).astype(np.float32)).astype(np.float32)
    return out


def forward_backward(params, X, y, casts=True):
    """Mean squared error of log(1+nnz) and its analytic gradient, in FP64.
    With casts, the weights and layer inputs are BF16-rounded in the forward
    pass and the roundings are treated as the identity in the backward pass."""
    p = np.asarray(params, np.float64)
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    if casts:
        wb = bf16_round(p.astype(np.float32)).astype(np.float64)
        cast = lambda a: bf16_round(a.astype(np.float32)).astype(np.float64)  # noqa: E731
    else:
        wb = p
        cast = lambda a: a  # noqa: E731
    W1, b1, W2, b2, W3, b3 = unpack(wb)
    x = cast(X)
    z1 = x @ W1.T + b1
    h1 = cast(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = cast(np.maximum(z2, 0.0))
    out = h2 @ W3 + b3
    n = len(y)
    err = out - y
    loss = float(np.mean(err * err))
    dout = 2.0 * err / n
    g = np.zeros(NPARAM)
    gW3 = h2.T @ dout
    gb3 = dout.sum()
    dz2 = np.outer(dout, W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    g[OFF_W1:OFF_B1] = gW1.ravel()
    g[OFF_B1:OFF_W2] = gb1
    g[OFF_W2:OFF_B2] = gW2.ravel()
    g[OFF_B2:OFF_W3] = gb2
    g[OFF_W3:OFF_B3] = gW3
    g[OFF_B3] = gb3
    return loss, g, out


def adam(params, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba); t is the 1-based step index."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def features(A_colptr, A_rowidx, B_colptr, B_rowidx, B_val, iteration, prev_nnz=None):
    """The 12 per-column input features, from their definitions:
    log1p nnz(B_*j), log1p flops_j, log1p max/mean/min nnz(A_*k) over k in
    B_*j, the iteration index, log1p of the row span of the product column,
    max_k b_kj, sum_k b_kj^2, log1p of the std of nnz(A_*k), log1p of the
    previous iteration's product nnz (0 if none), log1p sum_k b_kj nnz(A_*k)."""
    lenA = np.diff(np.asarray(A_colptr, np.int64))
    n = len(B_colptr) - 1
    F = np.zeros((n, 12), np.float64)
    for j in range(n):
        ks = B_rowidx[B_colptr[j]:B_colptr[j + 1]]
        bv = B_val[B_colptr[j]:B_colptr[j + 1]]
        L = lenA[ks].astype(np.float64)
        m = len(ks)
        fl = L.sum()
        nz = ks[L > 0]
        if len(nz):
            lo = min(A_rowidx[A_colptr[k]] for k in nz)
            hi = max(A_rowidx[A_colptr[k + 1] - 1] for k in nz)
            span = hi - lo + 1
        else:
            span = 0
        F[j] = [np.log1p(m), np.log1p(fl), np.log1p(L.max() if m else 0),
                np.log1p(fl / m if m else 0), np.log1p(L.min() if m else 0), iteration,
                np.log1p(span), bv.max() if m else 0, (bv * bv).sum(),
                np.log1p(L.std() if m else 0),
                np.log1p(prev_nnz[j]) if prev_nnz is not None else 0.0,
                np.log1p((bv * L).sum())]
    return F
