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
    """Features of the start of consecutive control steps of plain MPM
    rollouts and the targets (grid change over the step) after them, on the
    device, cropped to one box shape around each sample's material.

    The rollouts run in chunks of `chunk` scenes: a first pass records the
    stencil box of every scene at every control-step boundary (the box shape
    covers the material at the start and the end of every step, plus
    `margin` nodes), a second pass reruns them and keeps the crops, so only
    one chunk of whole-grid arrays is held at a time."""

    def __init__(self, scene_list: Sequence, n_blocks: int, crop: bool = True, margin: int = 4, chunk: int = 32):
        torch = _torch()
        S, R = len(scene_list), scene_list[0].res
        self.S, self.R, self.n_blocks = S, R, n_blocks
        chunk = max(1, min(int(chunk), S))
        shape = (R, R, R)
        if crop:
            boxes = []
            for c0 in range(0, S, chunk):
                boxes.append(self._boxes(scene_list[c0:c0 + chunk], n_blocks))
            bb = np.concatenate(boxes)
            shape = crop_shape(bb, margin, R)
        self.shape = shape
        D, H, W = shape
        with torch.cuda.device(0):
            self.feat = torch.zeros((n_blocks, S, D, H, W, CIN), dtype=torch.float32, device="cuda")
            self.target = torch.zeros((n_blocks, S, D, H, W, COUT), dtype=torch.float32, device="cuda")
            self.mask = torch.zeros((n_blocks, S, D, H, W), dtype=torch.float32, device="cuda")
        for c0 in range(0, S, chunk):
            self._fill(scene_list[c0:c0 + chunk], c0, n_blocks, crop)

    @staticmethod
    def _boxes(scenes_c, n_blocks):
        """[n][6] stencil boxes (inclusive) of every scene over every step of its rollout."""
        torch = _torch()
        sim = make_sim(scenes_c)
        n = len(scenes_c)
        out = np.zeros((n, 6), np.int64)
        out[:, :3], out[:, 3:] = 1 << 30, -1
        with torch.cuda.stream(sim.torch_stream):
            box = torch.zeros((n, 6), dtype=torch.int32, device="cuda")
            for b in range(n_blocks + 1):
                if b:
                    sim.step(SUBSTEPS)
                k = min(b, scenes_c[0].n_ctrl - 1)
                sim.set_colliders_ctrl(k)
                sim.sur_bbox(box)
                h = box.cpu().numpy()
                out[:, :3] = np.minimum(out[:, :3], h[:, :3])
                out[:, 3:] = np.maximum(out[:, 3:], h[:, 3:] + 1)   # one node past the stencil
        st = sim.sync()
        sim.close()
        if st < 0:
            raise RuntimeError(f"rollout failed ({st})")
        return out

    def _fill(self, scenes_c, s0, n_blocks, crop):
        torch = _torch()
        n, R = len(scenes_c), self.R
        sim = make_sim(scenes_c)
        with torch.cuda.stream(sim.torch_stream):
            feat = torch.zeros((n_blocks, n, R, R, R, CIN), dtype=torch.float32, device="cuda")
            target = torch.zeros((n_blocks, n, R, R, R, COUT), dtype=torch.float32, device="cuda")
            mask = torch.zeros((n_blocks, n, R, R, R), dtype=torch.float32, device="cuda")
            g_prev = torch.zeros((n, R, R, R, 4), dtype=torch.float32, device="cuda")
            g_next = torch.zeros_like(g_prev)
            f_next = torch.zeros((n, R, R, R, CIN), dtype=torch.float32, device="cuda")
            sim.set_colliders_ctrl(0)
            sim.sur_features(feat[0], g_prev)
            for b in range(n_blocks):
                sim.step(SUBSTEPS)
                k = min(b + 1, scenes_c[0].n_ctrl - 1)
                sim.set_colliders_ctrl(k)
                dst = feat[b + 1] if b + 1 < n_blocks else f_next
                sim.sur_features(dst, g_next)
                sim.sur_targets(g_prev, g_next, target[b], mask[b])
                g_prev, g_next = g_next, g_prev
            if not crop:
                self.feat[:, s0:s0 + n] = feat
                self.target[:, s0:s0 + n] = target
                self.mask[:, s0:s0 + n] = mask
            else:
                L = _unet_lib()
                st_ = sim.torch_stream.cuda_stream
                m = n_blocks * n
                box = torch.zeros((m, 6), dtype=torch.int32, device="cuda")
                origin = torch.zeros((m, 3), dtype=torch.int32, device="cuda")
                if L.mpm_nn_bbox(mask.data_ptr(), 1, m, R, box.data_ptr(), st_) != 0:
                    raise RuntimeError("mpm_nn_bbox failed")
                D, H, W = self.shape
                if L.mpm_nn_crop_origin(box.data_ptr(), m, R, D, H, W, origin.data_ptr(), st_) != 0:
                    raise RuntimeError("mpm_nn_crop_origin failed")
                for src, c, dst in ((feat, CIN, self.feat), (target, COUT, self.target), (mask, 1, self.mask)):
                    tmp = torch.zeros((m, D, H, W, c), dtype=torch.float32, device="cuda")
                    _crop_all(L, st_, src, c, m, R, origin, self.shape, tmp)
                    dst[:, s0:s0 + n] = tmp.view((n_blocks, n, D, H, W) + ((c,) if dst.dim() == 6 else ()))
        st = sim.sync()
        torch.cuda.synchronize()
        sim.close()
        if st < 0:
            raise RuntimeError(f"rollout failed ({st})")

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
          log_every: int = 50, holdout: Optional[RolloutData] = None, lr_final: Optional[float] = None,
          tail: float = 0.0) -> List[Dict]:
    """Adam on the masked MSE of the targets; returns a loss log.  With
    lr_final the step size falls from lr to lr_final on a cosine over the
    run; with tail > 0 it stays at lr and then falls linearly to lr / 20 over
    the last `tail` fraction of the steps (the weights at a constant step
    size keep wandering around the minimum; the last step decides which of
    them the network keeps)."""
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
        lr_t = lr
        if lr_final is not None:
            lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * (it - 1) / max(steps - 1, 1)))
        elif tail > 0.0:
            t0_tail = steps * (1.0 - tail)
            if it > t0_tail:
                lr_t = lr * (1.0 - 0.95 * (it - t0_tail) / max(steps - t0_tail, 1.0))
        loss = net.train_step(xb, tb.view(-1, COUT), mb.view(-1), lr=lr_t)
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
