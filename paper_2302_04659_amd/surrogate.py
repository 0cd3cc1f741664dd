"""Grid U-Net surrogate for one control step (25 substeps) of the batched
MLS-MPM, with the residual gate and per-scene plain-MPM fallback.

The paper has no learned component; this module adds one in front of the
substep loop of its soft-body simulator (Algorithm 1 runs 25 substeps per
control step, App. D.3).  Everything that computes runs in libmpm_hip.so:
feature extraction, the network (BF16 MFMA kernels), the particle advance,
the re-splat residual and the fallback (include/mpm.h, include/mpm_nn.h).
PyTorch only provides device buffers and the stream, and assembles training
batches by copying stored samples.

Network input (8 channels per node): mass and P2G momentum of the current
state, the clipped distance to the nearest collider and that collider's
velocity.  Output (4 channels): the change of the node velocity and mass
over the control step.  Training data come from plain MPM rollouts of the
slab-pushing workload (seeded scenes), generated on the device.
"""
from __future__ import annotations

import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import mpm as _mpm
from .unet import UNet

CIN, COUT = 8, 4
SUBSTEPS = 25


def _torch():
    import torch
    return torch


def make_sim(scene_list: Sequence):
    """A Sim on a fresh torch stream: the library's kernels, the network's
    kernels and the torch buffer work are then ordered on one stream."""
    torch = _torch()
    ts = torch.cuda.Stream()
    sim = _mpm.Sim(scene_list, stream=ts.cuda_stream)
    sim.torch_stream = ts
    return sim


def _stream_of(sim):
    torch = _torch()
    ts = getattr(sim, "torch_stream", None)
    if ts is None:
        if not sim.stream:
            raise ValueError("the Sim must run on a torch stream (create it with make_sim)")
        ts = torch.cuda.ExternalStream(sim.stream)
    return ts


class GridSurrogate:
    """Runs control steps of a Sim through a trained UNet.  Everything is
    queued on the Sim's stream."""

    def __init__(self, sim: "_mpm.Sim", net: UNet, threshold: float = 1e-3, chunk: int = 16):
        torch = _torch()
        self.sim, self.net, self.threshold, self.chunk = sim, net, float(threshold), int(chunk)
        self.ts = _stream_of(sim)
        R = sim.scenes[0].res
        S = sim.n_scenes
        dev = net.device
        self.R, self.S = R, S
        torch.cuda.synchronize()      # weights and buffers made on other streams are ready
        with torch.cuda.stream(self.ts):
            self.feat = torch.zeros((S, R, R, R, CIN), dtype=torch.float32, device=dev)
            self.grid0 = torch.zeros((S, R, R, R, 4), dtype=torch.float32, device=dev)
            self.pred = torch.zeros((S, R, R, R, COUT), dtype=torch.float32, device=dev)
            self.residual = torch.zeros(S, dtype=torch.float32, device=dev)
            self.n_fallback = torch.zeros(1, dtype=torch.int32, device=dev)

    def predict(self):
        """Features of the current state and the network's prediction (device)."""
        torch = _torch()
        with torch.cuda.stream(self.ts):
            self.sim.sur_features(self.feat, self.grid0)
            for i in range(0, self.S, self.chunk):
                j = min(self.S, i + self.chunk)
                self.net.forward(self.feat[i:j], out=self.pred[i:j])

    def block(self, fallback: bool = True, sync: bool = False):
        """One control step of every scene (surrogate, plain MPM where the
        residual is over the threshold)."""
        torch = _torch()
        self.predict()
        with torch.cuda.stream(self.ts):
            self.sim.sur_block(self.pred, self.grid0, self.threshold, fallback=fallback, sync=sync,
                               residual=self.residual, n_fallback=self.n_fallback)

    def block_with(self, pred, fallback: bool = False):
        """A control step from a given prediction (baselines)."""
        torch = _torch()
        with torch.cuda.stream(self.ts):
            self.sim.sur_features(self.feat, self.grid0)
            self.sim.sur_block(pred, self.grid0, self.threshold, fallback=fallback, residual=self.residual,
                               n_fallback=self.n_fallback)


# ---------------------------------------------------------------------- data
class RolloutData:
    """Start grids and features of consecutive control steps of plain MPM
    rollouts, and the targets between them (all on the device)."""

    def __init__(self, scene_list: Sequence, n_blocks: int):
        torch = _torch()
        sim = make_sim(scene_list)
        S, R = sim.n_scenes, scene_list[0].res
        self.S, self.R, self.n_blocks = S, R, n_blocks
        with torch.cuda.stream(sim.torch_stream):
            self.feat = torch.zeros((n_blocks, S, R, R, R, CIN), dtype=torch.float32, device="cuda")
            self.target = torch.zeros((n_blocks, S, R, R, R, COUT), dtype=torch.float32, device="cuda")
            self.mask = torch.zeros((n_blocks, S, R, R, R), dtype=torch.float32, device="cuda")
            g_prev = torch.zeros((S, R, R, R, 4), dtype=torch.float32, device="cuda")
            g_next = torch.zeros_like(g_prev)
            f_next = torch.zeros((S, R, R, R, CIN), dtype=torch.float32, device="cuda")
            sim.set_colliders_ctrl(0)
            sim.sur_features(self.feat[0], g_prev)
            for b in range(n_blocks):
                sim.step(SUBSTEPS)
                k = min(b + 1, scene_list[0].n_ctrl - 1)
                sim.set_colliders_ctrl(k)
                dst = self.feat[b + 1] if b + 1 < n_blocks else f_next
                sim.sur_features(dst, g_next)
                sim.sur_targets(g_prev, g_next, self.target[b], self.mask[b])
                g_prev, g_next = g_next, g_prev
        st = sim.sync()
        torch.cuda.synchronize()
        if st < 0:
            raise RuntimeError(f"rollout failed ({st})")
        sim.close()

    @property
    def n_samples(self):
        return self.n_blocks * self.S

    def batch(self, idx, xb, tb, mb):
        for j, k in enumerate(idx):
            b, s = divmod(int(k), self.S)
            xb[j].copy_(self.feat[b, s])
            tb[j].copy_(self.target[b, s])
            mb[j].copy_(self.mask[b, s])


def train(net: UNet, data: RolloutData, steps: int, batch: int = 8, lr: float = 3e-4, seed: int = 0,
          log_every: int = 50, holdout: Optional[RolloutData] = None) -> List[Dict]:
    """Adam on the masked MSE of the targets; returns a loss log."""
    torch = _torch()
    R = data.R
    rng = np.random.default_rng(seed)
    xb = torch.zeros((batch, R, R, R, CIN), dtype=torch.float32, device="cuda")
    tb = torch.zeros((batch, R, R, R, COUT), dtype=torch.float32, device="cuda")
    mb = torch.zeros((batch, R, R, R), dtype=torch.float32, device="cuda")
    log = []
    t0 = time.perf_counter()
    for it in range(1, steps + 1):
        idx = rng.choice(data.n_samples, size=batch, replace=False)
        data.batch(idx, xb, tb, mb)
        loss = net.train_step(xb, tb.view(-1, COUT), mb.view(-1), lr=lr)
        if it % log_every == 0 or it == steps:
            rec = {"step": it, "loss": loss.value(), "s": time.perf_counter() - t0}
            if holdout is not None:
                rec["holdout_loss"] = evaluate_loss(net, holdout, batch)
            log.append(rec)
            print("[train]", rec, file=sys.stderr, flush=True)
    return log


def evaluate_loss(net: UNet, data: RolloutData, batch: int = 8) -> float:
    """Masked MSE over every sample of `data` (forward only)."""
    torch = _torch()
    R = data.R
    xb = torch.zeros((batch, R, R, R, CIN), dtype=torch.float32, device="cuda")
    tb = torch.zeros((batch, R, R, R, COUT), dtype=torch.float32, device="cuda")
    mb = torch.zeros((batch, R, R, R), dtype=torch.float32, device="cuda")
    tot, n = 0.0, 0
    for i in range(0, data.n_samples - batch + 1, batch):
        data.batch(range(i, i + batch), xb, tb, mb)
        pred = net.forward(xb)
        loss, _ = net.loss_and_grad(pred, tb.view(-1, COUT), mb.view(-1))
        tot += loss.value()
        n += 1
    return tot / max(n, 1)
