"""Learned output-size estimator: data collection from the method's own runs,
training with the library's MLP kernels, and storage of the packed weights.

Rows are (12 per-column features, log(1 + exact product nnz)) logged at every
MCL iteration of training graphs: the features come from the symbolic pass
(`mcl_estimate(..., features)`), the exact nnz from the fused iteration
(`mcl_params.nnz_out`).  Training runs `mcl_mlp_train_step` (forward,
backward and Adam on the GPU) over shuffled mini-batches.
"""
from __future__ import annotations

import os
import time

import numpy as np
import torch

from . import mcl

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "mlp_weights.npy")


def collect(A: "mcl.DeviceCSC", iterations: int = 4, params=None, log=None):
    """Run `iterations` MCL iterations from A; return (features, targets) on the GPU."""
    feats, targs = [], []
    for it in range(iterations):
        _, F = mcl.estimate(A, A, features=True, estimator=mcl.EST_COHEN, iteration=it)
        nnz = torch.empty(A.ncols, dtype=torch.int64, device="cuda")
        An, change, st = mcl.iterate(A, params, nnz_out=nnz, iteration=it)
        F = F.clone()
        F[:, 5] = float(it)
        feats.append(F)
        targs.append(torch.log1p(nnz.double()).float())
        if log:
            log("collect it=%d cols=%d change=%.3g" % (it, A.ncols, change))
        A = An
        if change < 1e-9:
            break
    return torch.cat(feats), torch.cat(targs)


def train(X: torch.Tensor, y: torch.Tensor, epochs: int = 4, batch: int = 65536, lr: float = 2e-3,
          seed: int = 0, log=None):
    """Train from scratch with the GPU kernels; returns (state, packed, losses)."""
    state, packed = mcl.mlp_init(seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = y.numel()
    losses = []
    t = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        el = []
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            if idx.numel() < 256:
                continue
            lr_t = lr * (0.5 ** ep)
            el.append(mcl.mlp_train_step(state, packed, X[idx].contiguous(), y[idx].contiguous(),
                                         lr=lr_t))
        losses.append(float(np.mean(el)))
        if log:
            log("epoch %d loss %.4f (%.1f s)" % (ep, losses[-1], time.time() - t))
    return state, packed, losses


def save(packed: torch.Tensor, path: str = WEIGHTS):
    np.save(path, packed.cpu().numpy())


def load(path: str = WEIGHTS):
    if not os.path.exists(path):
        return None
    return torch.from_numpy(np.load(path)).cuda()


def evaluate(packed, A: "mcl.DeviceCSC", iteration: int = 0):
    """Median and p99 of |log est - log nnz| for the learned and Cohen estimators."""
    nnz = torch.empty(A.ncols, dtype=torch.int64, device="cuda")
    mcl.iterate(A, nnz_out=nnz, iteration=iteration)
    out = {}
    for name, kw in (("mlp", dict(estimator=mcl.EST_MLP, mlp_weights=packed)),
                     ("cohen", dict(estimator=mcl.EST_COHEN))):
        est = mcl.estimate(A, A, iteration=iteration, **kw)
        err = torch.abs(torch.log1p(est.double()) - torch.log1p(nnz.double()))
        big = nnz > 768
        out[name] = dict(median=float(err.median()), p99=float(torch.quantile(err[::7], 0.99)),
                         median_big=float(err[big].median()) if big.any() else 0.0)
    return out
