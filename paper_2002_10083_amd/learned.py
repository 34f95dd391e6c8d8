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


def residual_quantiles(A: "mcl.DeviceCSC", est_kw: dict, iterations: int = 2, params=None,
                       qs=(0.5, 0.75, 0.9, 0.95, 0.99), min_est: float = 384.0):
    """Quantiles of log(nnz) - log(estimate) over the columns an estimator
    sizes (estimate above `min_est`; smaller columns are planned by their
    exact-safe bound), pooled over the first `iterations` MCL iterations of A."""
    res = []
    for it in range(iterations):
        nnz = torch.empty(A.ncols, dtype=torch.int64, device="cuda")
        An, change, _ = mcl.iterate(A, params, nnz_out=nnz, iteration=it)
        est = mcl.estimate(A, A, iteration=it, **est_kw)
        m = est > min_est
        res.append((torch.log(nnz.double().clamp(min=1)) - torch.log(est.double().clamp(min=1)))[m])
        A = An
        if change < 1e-9:
            break
    r = torch.cat(res).float()
    if r.numel() > (1 << 24):  # torch.quantile's input limit
        r = r[torch.randperm(r.numel(), device=r.device)[:1 << 24]]
    q = torch.quantile(r, torch.tensor(list(qs), device=r.device))
    return {float(k): float(v) for k, v in zip(qs, q)}


#: the planner sizes a column for 1.3 * est_scale * estimate keys
PLAN_MARGIN = 1.3


def scale_for_quantile(quantiles: dict, q: float = 0.75) -> float:
    """est_scale that sizes every column for exp(Q_q) times its estimate,
    Q_q the q-quantile of the log residual on held-out graphs."""
    return float(np.exp(quantiles[q]) / PLAN_MARGIN)


def train(X: torch.Tensor, y: torch.Tensor, epochs: int = 4, batch: int = 65536, lr: float = 2e-3,
          seed: int = 0, log=None, decay: float = 0.5):
    """Train from scratch with the GPU kernels (learning rate lr * decay**epoch);
    returns (state, packed, losses)."""
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
            lr_t = lr * (decay ** ep)
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
