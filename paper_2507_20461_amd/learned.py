"""Learned GENO gate: harvest, training and choice of the gate margin.

Every numerical step runs in the library's kernels (harvest, forward and
backward passes, Adam, bfloat16 inference); this module only orders the
calls, slices minibatches and keeps the bookkeeping.

Recipe (the gate's reading of the method):
* harvest per cell and direction the normalised 5-cell stencil and the
  smallest plain-GENO chi of the cell's two face-sides (geno_harvest) from
  solver runs: the seeded 2-D quadrant grids, and the 1-D sine and jump runs
  embedded as y-invariant 2-D grids (4 rows, periodic in y);
* stratify so that stencils with chi < 0.999 make up at least 20 % of the set;
* train with the mean binary cross-entropy, Adam, float32 master weights;
* choose delta on held-out stencils: the largest candidate whose misgate rate
  (gate on, chi < 0.999) stays at most 1e-4 of the held-out set.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import geno_gks as G
from . import inputs

NIN, NH, NPARAM = 40, 64, 6849
CHI_SMOOTH = 0.999


def init_params(seed, device="cuda"):
    """He-scaled normal weights, zero biases (W1, b1, W2, b2, w3, b3)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((NH, NIN)) * math.sqrt(2.0 / NIN)
    W2 = rng.standard_normal((NH, NH)) * math.sqrt(2.0 / NH)
    w3 = rng.standard_normal(NH) * math.sqrt(1.0 / NH)
    p = np.concatenate([W1.ravel(), np.zeros(NH), W2.ravel(), np.zeros(NH), w3, [0.0]])
    return torch.tensor(p, dtype=torch.float32, device=device)


def _harvest_run(grid, W, dW, steps, every, out):
    """Runs the solver and harvests both directions every `every` steps."""
    Wd, dWd = grid.to_device(W), grid.grad_to_device(dW)
    ws = grid.workspace()
    done = 0
    while True:
        for d in (0, 1) if grid.ny > 4 else (0,):
            X, y = G.harvest(grid, Wd, dWd, ws, d)
            out.append((X, y))
        if done >= steps:
            break
        n = min(every, steps - done)
        G.gks_step(grid, Wd, dWd, ws, n)
        done += n


def _embed_1d(W1, dW1, rows=4):
    """y-invariant 2-D copy of a 1-D state (rhoV = 0, d/dy = 0)."""
    nx = W1.shape[2]
    W = np.zeros((4, rows, nx))
    W[0], W[1], W[3] = W1[0, 0], W1[1, 0], W1[2, 0]
    dW = np.zeros((8, rows, nx))
    dW[0], dW[1], dW[3] = dW1[0, 0], dW1[1, 0], dW1[2, 0]
    return W, dW


def harvest_dataset(n2d=512, seeds=(0, 1, 2, 3), steps=100, every=5):
    """Stencils and targets from the quadrant grids (n2d^2, one run per seed)
    and the 1-D runs (200 cells, 200 steps). Returns float32 device tensors."""
    parts = []
    for s in seeds:
        W, dW, _ = inputs.quadrants_2d(n2d, n2d, s)
        _harvest_run(G.Grid(2, n2d, n2d, bc=G.BC_TRANSMISSIVE), W, dW, steps, every, parts)
    W1, dW1 = inputs.sine_1d(200)
    W, dW = _embed_1d(W1, dW1)
    _harvest_run(G.Grid(2, 200, 4, bc=G.BC_PERIODIC), W, dW, 200, 10, parts)
    for s in range(5):
        W1, dW1, _ = inputs.jump_1d(200, s)
        W, dW = _embed_1d(W1, dW1)
        g = G.Grid(2, 200, 4, bc=(G.BC_TRANSMISSIVE, G.BC_TRANSMISSIVE, G.BC_PERIODIC, G.BC_PERIODIC))
        _harvest_run(g, W, dW, 200, 10, parts)
    X = torch.cat([p[0] for p in parts])
    y = torch.cat([p[1] for p in parts])
    return X, y


def stratify(X, y, seed=0, frac_rough=0.2):
    """All stencils with chi < CHI_SMOOTH and as many smooth ones as keep the
    rough share >= frac_rough (shuffled)."""
    g = torch.Generator(device=X.device).manual_seed(seed)
    rough = torch.nonzero(y < CHI_SMOOTH).flatten()
    smooth = torch.nonzero(y >= CHI_SMOOTH).flatten()
    keep = min(smooth.numel(), int(rough.numel() * (1.0 - frac_rough) / frac_rough))
    smooth = smooth[torch.randperm(smooth.numel(), generator=g, device=X.device)[:keep]]
    idx = torch.cat([rough, smooth])
    idx = idx[torch.randperm(idx.numel(), generator=g, device=X.device)]
    return X[idx].contiguous(), y[idx].contiguous()


def train(X, y, epochs=2, batch=8192, lr=2e-3, seed=0, log=None):
    """Adam on minibatches (library kernels). Returns (params, losses per epoch)."""
    dev = X.device
    p = init_params(seed, dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    grad = torch.empty_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = G.mlp_train_workspace(batch, dev)
    n = X.shape[0]
    t = 0
    hist = []
    gen = torch.Generator(device=dev).manual_seed(seed + 1)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=dev)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            Xb, yb = X[idx].contiguous(), y[idx].contiguous()
            G.mlp_grad(p, Xb, yb, grad, loss, ws)
            t += 1
            G.mlp_adam(p, grad, m, v, t, lr * (0.5 if ep == epochs - 1 and epochs > 1 else 1.0))
            if b0 % (64 * batch) == 0:
                tot += float(loss.item())
                cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log("epoch %d: mean sampled loss %.5f" % (ep, hist[-1]))
    return p, hist


def choose_delta(prob, y, candidates=(0.3, 0.1, 0.03, 0.01, 3e-3, 1e-3, 3e-4, 1e-4), max_misgate=1e-4):
    """Largest delta whose misgate rate (gate on while chi < CHI_SMOOTH) is at
    most max_misgate of the held-out set; also the share of gated stencils."""
    rough = y < CHI_SMOOTH
    n = y.numel()
    for d in candidates:
        on = prob >= 1.0 - d
        mis = float((on & rough).sum()) / n
        if mis <= max_misgate:
            return d, {"delta": d, "misgate": mis, "gated": float(on.sum()) / n}
    return 0.0, {"delta": 0.0, "misgate": 0.0, "gated": 0.0}
