"""Training pipeline of the learned basis-function surrogate.

Patches are produced by the method itself: an FP64 solve of each given
problem and mobility, then the library's input builder (log mobility and
skeleton masks) and target builder (the normalised basis functions of that
solve).  The network is trained by the library's BF16 forward/backward and
Adam kernels (SurrogateNet.train_step); this module only orders the calls.
"""
from __future__ import annotations

import time

import numpy as np

from .mrcm import MRCMSolver, SurrogateNet


def method_patches(cases):
    """Inputs and targets of every subdomain of every (problem, saturation)
    case, from FP64 solves on the GPU: torch device tensors
    ([N, 256, 8] bfloat16, [N, 256, 16] float32)."""
    import torch
    xs, ys = [], []
    sol, cur = None, None
    try:
        for prob, sat in cases:
            if prob is not cur:          # one setup per problem, several mobilities
                if sol is not None:
                    sol.close()
                sol, cur = MRCMSolver(prob, precision="fp64"), prob
            sol.update_mobility(sat if sat is not None else np.ones(prob.nx * prob.ny), sat is None)
            sol.solve()
            xs.append(sol.surrogate_inputs())
            ys.append(sol.surrogate_targets())
    finally:
        if sol is not None:
            sol.close()
    return torch.cat(xs), torch.cat(ys)


def train(net: SurrogateNet, x, y, steps: int, batch: int, lr: float = 1e-3, seed: int = 0,
          lr_final: float | None = None, time_limit: float | None = None):
    """Adam on random mini-batches of (x, y) for `steps` steps (or until
    `time_limit` seconds); the learning rate decays geometrically to
    lr_final when given.  Returns the per-step batch losses."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = x.shape[0]
    batch = min(batch, n, net.max_batch)
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        idx = torch.randint(0, n, (batch,), generator=gen).to(x.device)
        xb, yb = x.index_select(0, idx).contiguous(), y.index_select(0, idx).contiguous()
        rate = lr if lr_final is None else lr * (lr_final / lr) ** (k / max(steps - 1, 1))
        losses.append(net.train_step(xb, yb, rate))
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
    return np.array(losses)


def evaluate(net: SurrogateNet, x, y, batch: int | None = None) -> float:
    """Mean squared error of the network on (x, y)."""
    batch = batch or net.max_batch
    tot, n = 0.0, 0
    for i in range(0, x.shape[0], batch):
        xb, yb = x[i:i + batch].contiguous(), y[i:i + batch].contiguous()
        loss, _ = net.loss_grad(xb, yb)
        tot += loss * xb.shape[0]
        n += xb.shape[0]
    return tot / max(n, 1)
