"""Training pairs and training of the learned warm start of the Poisson solve.

Pairs come from the library itself: a simulation instance is loaded with a
seeded particle load, stepped, and its potential solved to a tight tolerance;
pic_training_sample then writes x = q / s and the dimensionless charge
response y (see include/pic.h). Training runs forward, backward and Adam in
the library's kernels; this module only orders the calls.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import pic
from . import workloads as W


def collect_samples(base: W.Config, fields, per_field: int, steps_between: int, counts, region="near_tip",
                    kT_eV=None, caps=None, seed=11, solve_rtol=1e-12, device="cuda", log_every: int = 500):
    """(x, y) pairs as fp32 device tensors of shape [nz][ny][nx]: for each apex
    field, a fresh instance with its own load, sampled every steps_between
    full steps after a solve to solve_rtol."""
    nz, ny, nx = base.nz, base.ny, base.nx
    xs, ys = [], []
    if caps is None:
        caps = (4 * counts[0] + 65536, 4 * counts[1] + 65536, counts[2] + 4096)
    for i, F in enumerate(fields):
        cfg = dataclasses.replace(base, apex_field=float(F), seed=seed + 97 * i)
        sim = pic.Simulation(cfg, caps=caps, precision=pic.PIC_F64, solver=pic.PIC_SOLVER_MGCG, device=device,
                             step_rtol=1e-10)
        try:
            sim.load(W.initial_load(cfg, counts=counts, kT_eV=kT_eV, region=region, seed=seed + 13 * i))
            sim.step(1, pic.STEP_DEPOSIT)
            for k in range(per_field):
                if k or steps_between == 0:
                    sim.step(max(steps_between, 1), pic.STEP_FULL)
                sim.solve(solver=pic.PIC_SOLVER_MGCG, guess=pic.PIC_GUESS_PREVIOUS, rtol=solve_rtol, maxit=100000)
                x = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
                y = torch.empty_like(x)
                torch.cuda.synchronize(device)
                pic.pic_training_sample(sim.ctx, x.data_ptr(), y.data_ptr())
                torch.cuda.synchronize(device)
                xs.append(x)
                ys.append(y)
                if log_every and k % log_every == log_every - 1:
                    print(f"[warmstart] field {F / 1e9:.1f} GV/m: {k + 1} pairs", flush=True)
        finally:
            sim.close()
    return torch.stack(xs), torch.stack(ys)


def train(net: pic.UNet, X: torch.Tensor, Y: torch.Tensor, iters: int, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, lr_final: float | None = None, normalize: bool = True):
    """Adam on random mini-batches (of the network's batch size) of the pairs;
    returns the losses of every step (of the normalized targets). With
    lr_final the rate decays geometrically from lr to lr_final. With
    normalize the targets are divided by their RMS during training and the
    linear head is scaled by it afterwards, so the network outputs y itself."""
    B = net.shape[0]
    rng = np.random.default_rng(seed)
    sY = float(Y.pow(2).mean().sqrt()) if normalize else 1.0
    if not sY > 0:
        sY = 1.0
    Yn = Y / sY
    losses = []
    for it in range(iters):
        idx = torch.as_tensor(rng.choice(X.shape[0], size=B, replace=X.shape[0] < B), device=X.device)
        r = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(iters - 1, 1))
        loss = net.train_step(X[idx], Yn[idx], r, want_loss=True)
        losses.append(loss)
        if log_every and it % log_every == 0:
            print(f"[warmstart] iter {it} loss {loss:.4e}", flush=True)
    if sY != 1.0:
        # head = last (base + 1) parameters: w[base], b
        nh = net.cfg.base_channels + 1
        torch.cuda.synchronize(net.device)
        net.params[-nh:] *= sY
        torch.cuda.synchronize(net.device)
        net.sync()
    return losses
