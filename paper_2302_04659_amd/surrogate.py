"""Grid U-Net surrogate for one control step (25 substeps) of the batched
MLS-MPM, with the residual gate and per-scene plain-MPM fallback.

The paper has no learned component; this module adds one in front of the
substep loop of its soft-body simulator (Algorithm 1 runs 25 substeps per
control step, App. E.3).  Everything that computes runs in libmpm_hip.so:
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
from .unet import nn_lib as _unet_lib

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


def crop_shape(bbox: np.ndarray, margin: int, R: int):
    """Common crop size of a batch: the largest material extent plus a margin
    on each side, rounded up to a multiple of 8 and at most R."""
    ext = (bbox[:, 3:] - bbox[:, :3]).max(axis=0) + 2 * margin
    return tuple(int(min(R, max(8, -(-e // 8) * 8))) for e in ext)


def _crop_all(L, stream, src, c, n, R, origin, shape, dst, uncrop=0):
    D, H, W = shape
    r = L.mpm_nn_crop(src.data_ptr(), c, n, R, origin.data_ptr(), D, H, W, dst.data_ptr(), uncrop, stream)
    if r != 0:
        raise RuntimeError(f"mpm_nn_crop failed ({r})")


class GridSurrogate:
    """Runs control steps of a Sim through a trained UNet.  Everything is
    queued on the Sim's stream."""

    def __init__(self, sim: "_mpm.Sim", net: UNet, threshold: float = 1e-3, chunk: int = 0, margin: int = 4,
                 crop: bool = True):
        torch = _torch()
        # scenes per network launch (0: all at once -- the coarse levels of a crop are small, and only
        # a large batch fills the GPU; activations take ~1 KB per crop voxel)
        self.sim, self.net, self.threshold = sim, net, float(threshold)
        self.chunk = int(chunk) if chunk > 0 else sim.n_scenes
        self.margin, self.crop = int(margin), bool(crop)
        self.ts = _stream_of(sim)
        R = sim.scenes[0].res
        S = sim.n_scenes
        dev = net.device
        self.R, self.S = R, S
        self.crop_shape = (R, R, R)
        self._cbuf = None
        torch.cuda.synchronize()      # weights and buffers made on other streams are ready
        with torch.cuda.stream(self.ts):
            self.residual = torch.zeros(S, dtype=torch.float32, device=dev)
            self.n_fallback = torch.zeros(1, dtype=torch.int32, device=dev)
            self.box = torch.zeros((S, 6), dtype=torch.int32, device=dev)
            self.origin = torch.zeros((S, 3), dtype=torch.int32, device=dev)
        self._dense = None            # whole-grid arrays (crop = False, block_with), made on first use
        self._cur = None              # (prediction, start grid, box origin or None) of the last predict()

    def dense(self):
        """Whole-grid feat, grid0 and pred arrays (made on first use)."""
        torch = _torch()
        if self._dense is None:
            S, R, dev = self.S, self.R, self.net.device
            with torch.cuda.stream(self.ts):
                self._dense = (torch.zeros((S, R, R, R, CIN), dtype=torch.float32, device=dev),
                               torch.zeros((S, R, R, R, 4), dtype=torch.float32, device=dev),
                               torch.zeros((S, R, R, R, COUT), dtype=torch.float32, device=dev))
        return self._dense

    def predict(self):
        """Features of the current state and the network's prediction (device).
        With crop = True the features are made and the network runs on a box
        around each scene's material (the nodes the particles' P2G stencils
        reach, plus a margin; one host read of the boxes per call), and the
        prediction is zero outside it."""
        torch = _torch()
        L = self.net.L
        with torch.cuda.stream(self.ts):
            s = self.ts.cuda_stream
            if not self.crop:
                feat, grid0, pred = self.dense()
                self.sim.sur_features(feat, grid0)
                for i in range(0, self.S, self.chunk):
                    j = min(self.S, i + self.chunk)
                    self.net.forward(feat[i:j], out=pred[i:j])
                self._cur = (pred, grid0, None)
                return
            self.sim.sur_bbox(self.box)
            shape = crop_shape(self.box.cpu().numpy(), self.margin, self.R)
            D, H, W = shape
            if L.mpm_nn_crop_origin(self.box.data_ptr(), self.S, self.R, D, H, W, self.origin.data_ptr(), s) != 0:
                raise RuntimeError("mpm_nn_crop_origin failed")
            if self._cbuf is None or self._cbuf[0] != shape:
                dev = self.net.device
                self._cbuf = (shape,
                              torch.zeros((self.S, D, H, W, CIN), dtype=torch.float32, device=dev),
                              torch.zeros((self.S, D, H, W, 4), dtype=torch.float32, device=dev),
                              torch.zeros((self.S, D, H, W, COUT), dtype=torch.float32, device=dev))
            _, fc, gc, pc = self._cbuf
            self.crop_shape = shape
            self.sim.sur_features(fc, gc, origin=self.origin)
            for i in range(0, self.S, self.chunk):
                j = min(self.S, i + self.chunk)
                self.net.forward(fc[i:j], out=pc[i:j])
            self._cur = (pc, gc, self.origin)

    def block(self, fallback: bool = True, sync: bool = False):
        """One control step of every scene (surrogate, plain MPM where the
        residual is over the threshold)."""
        torch = _torch()
        self.predict()
        pred, grid0, origin = self._cur
        with torch.cuda.stream(self.ts):
            self.sim.sur_block(pred, grid0, self.threshold, fallback=fallback, sync=sync,
                               residual=self.residual, n_fallback=self.n_fallback, origin=origin)

    def block_with(self, pred, fallback: bool = False):
        """A control step from a given whole-grid prediction (baselines)."""
        torch = _torch()
        feat, grid0, _ = self.dense()
        with torch.cuda.stream(self.ts):
            self.sim.sur_features(feat, grid0)
            self.sim.sur_block(pred, grid0, self.threshold, fallback=fallback, residual=self.residual,
                               n_fallback=self.n_fallback)


# ---------------------------------------------------------------------- data
class RolloutData:
    """Start grids and features of consecutive control steps of plain MPM
    rollouts, and the targets between them (all on the device)."""

    def __init__(self, scene_list: Sequence, n_blocks: int, crop: bool = True, margin: int = 4):
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
        self.shape = (R, R, R)
        if crop:
            self._crop(margin)

    def _crop(self, margin: int):
        """Keep a box around each sample's material (start or end of the
        step): the network trains on the same kind of crop it runs on."""
        torch = _torch()
        L = _unet_lib()
        n, R = self.n_blocks * self.S, self.R
        s = torch.cuda.current_stream().cuda_stream
        box = torch.zeros((n, 6), dtype=torch.int32, device="cuda")
        origin = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
        if L.mpm_nn_bbox(self.mask.data_ptr(), 1, n, R, box.data_ptr(), s) != 0:
            raise RuntimeError("mpm_nn_bbox failed")
        shape = crop_shape(box.cpu().numpy(), margin, R)
        D, H, W = shape
        if L.mpm_nn_crop_origin(box.data_ptr(), n, R, D, H, W, origin.data_ptr(), s) != 0:
            raise RuntimeError("mpm_nn_crop_origin failed")
        out = []
        for src, c in ((self.feat, CIN), (self.target, COUT), (self.mask, 1)):
            dst = torch.zeros((n, D, H, W, c), dtype=torch.float32, device="cuda")
            _crop_all(L, s, src, c, n, R, origin, shape, dst)
            out.append(dst)
        torch.cuda.synchronize()
        self.feat = out[0].view(self.n_blocks, self.S, D, H, W, CIN)
        self.target = out[1].view(self.n_blocks, self.S, D, H, W, COUT)
        self.mask = out[2].view(self.n_blocks, self.S, D, H, W)
        self.shape = shape

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
    sh = tuple(data.shape)
    rng = np.random.default_rng(seed)
    xb = torch.zeros((batch,) + sh + (CIN,), dtype=torch.float32, device="cuda")
    tb = torch.zeros((batch,) + sh + (COUT,), dtype=torch.float32, device="cuda")
    mb = torch.zeros((batch,) + sh, dtype=torch.float32, device="cuda")
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
    sh = tuple(data.shape)
    xb = torch.zeros((batch,) + sh + (CIN,), dtype=torch.float32, device="cuda")
    tb = torch.zeros((batch,) + sh + (COUT,), dtype=torch.float32, device="cuda")
    mb = torch.zeros((batch,) + sh, dtype=torch.float32, device="cuda")
    tot, n = 0.0, 0
    for i in range(0, data.n_samples - batch + 1, batch):
        data.batch(range(i, i + batch), xb, tb, mb)
        pred = net.forward(xb)
        loss, _ = net.loss_and_grad(pred, tb.view(-1, COUT), mb.view(-1))
        tot += loss.value()
        n += 1
    return tot / max(n, 1)
