"""Learned proposal (not part of the paper's method): log frontier records
from plain runs, train the network on the GPU, and bound with it.

The network predicts, from 16 features of a frontier triangle, how far above
its largest vertex distance the maximum distance to B over the triangle lies
(in units of its longest edge). The engine uses the prediction to take the
sub-batch of each round in order of predicted maximum distance (so that the
lower bound rises early) and, in mode 2, to skip u3 and u4 for triangles it
predicts to stay active. Discards and the certificate still come only from
the rigorous bounds.

Every step runs in the library's kernels; this module only moves tensors and
draws the random numbers the training consumes (initial weights, minibatch
order), seeded.
"""
from __future__ import annotations

import numpy as np

from . import (PREC_FP32_RECHECK, bound, bound_batched, build_bvh, build_bvh_batched, mlp_forward, mlp_nparams,
               mlp_train)

NIN, NH = 16, 64


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal hidden layers, a small output layer, zero biases (FP32)."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2.0 / NIN), NIN * NH), np.zeros(NH),
             rng.normal(0, np.sqrt(2.0 / NH), NH * NH), np.zeros(NH),
             rng.normal(0, np.sqrt(1.0 / NH), NH), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == mlp_nparams()
    return p


def _cu(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def log_frontier(workloads, subbatch: int = 0, cap: int = 1 << 20, precision=PREC_FP32_RECHECK):
    """Run the plain method with the frontier log on; return the logged rows
    (features, label) of every workload, rows of too-deep parents dropped.
    A workload is (VA, FA, VB, FB, eps) or a list of them (one batched call)."""
    import torch
    out = []
    for W in workloads:
        log = torch.empty((cap, 17), dtype=torch.float32, device="cuda")
        if isinstance(W, list):
            bvh = build_bvh_batched([(_cu(VB, torch), _cu(FB, torch)) for _, _, VB, FB, _ in W])
            _, _, st = bound_batched([(_cu(VA, torch), _cu(FA, torch)) for VA, FA, _, _, _ in W], bvh,
                                     [e for *_, e in W], precision=precision, subbatch=subbatch, log_out=log, relative=True)
        else:
            VA, FA, VB, FB, eps = W
            bvh = build_bvh(_cu(VB, torch), _cu(FB, torch))
            _, _, st = bound(_cu(VA, torch), _cu(FA, torch), bvh, eps, precision=precision, subbatch=subbatch,
                             log_out=log, relative=True)
        rows = log[:st["logged"]].cpu().numpy()
        out.append(rows[np.all(np.isfinite(rows), 1)])
    return np.concatenate(out) if out else np.zeros((0, 17), np.float32)


def train(rows: np.ndarray, epochs: int = 8, batch: int = 512, lr: float = 2e-3, seed: int = 0):
    """Adam on the GPU over the logged rows; returns (params tensor, minibatch
    losses). 1/16 of the rows (seeded) are held out and their loss before and
    after training is returned too."""
    import torch
    rng = np.random.default_rng(seed)
    n = rows.shape[0]
    perm = rng.permutation(n)
    nval = max(1, n // 16)
    val, tr = perm[:nval], perm[nval:]
    X = _cu(rows[:, :16].astype(np.float32), torch)
    t = _cu(rows[:, 16].astype(np.float32), torch)
    P = _cu(init_params(seed), torch)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)

    def val_loss():
        y = mlp_forward(X[_cu(val, torch)], P)
        return float(((y - t[_cu(val, torch)]) ** 2).mean())

    before = val_loss()
    steps_per_epoch = max(1, tr.size // batch)
    order = np.concatenate([rng.permutation(tr)[:steps_per_epoch * batch] for _ in range(epochs)]).astype(np.int32)
    losses = mlp_train(X, t, _cu(order, torch), batch, P, M, V, step0=0, lr=lr)
    return P, losses.cpu().numpy(), (before, val_loss())
