"""Grid U-Net surrogate on the library's BF16-MFMA kernels (include/mpm_nn.h).

The network graph (which kernel runs on which buffer) lives here; every
arithmetic step is a launch of a kernel of libmpm_hip.so.  PyTorch only
allocates device memory and supplies the stream.

Architecture (3 levels, 32/64/128 channels, 3^3 convolutions):
  e1a, e1b: conv3 + ReLU at R^3            d1: 2^3 stride 2 -> 64 ch
  e2a, e2b: conv3 + ReLU at (R/2)^3        d2: 2^3 stride 2 -> 128 ch
  e3a, e3b: conv3 + ReLU at (R/4)^3
  u2: nearest x2 + conv3 -> 64, concat e2b, c2a, c2b
  u1: nearest x2 + conv3 -> 32, concat e1b, c1a, c1b
  head: 1^3 conv -> output channels
Weights are FP32 masters [taps][cin][cout]; BF16 packed copies feed the
MFMA kernels and are refreshed after each optimiser step.
"""
from __future__ import annotations

import ctypes as ct
import math
from typing import Dict, Optional

import numpy as np

from . import mpm as _mpm

KIND = {"c3": 0, "up": 1, "down": 2, "c1": 3}
TAPS = {"c3": 27, "up": 27, "down": 8, "c1": 1}

# name, kind, cin, cout, relu (cin None = network input, padded to 16)
LAYERS = [
    ("e1a", "c3", None, 32, True), ("e1b", "c3", 32, 32, True), ("d1", "down", 32, 64, True),
    ("e2a", "c3", 64, 64, True), ("e2b", "c3", 64, 64, True), ("d2", "down", 64, 128, True),
    ("e3a", "c3", 128, 128, True), ("e3b", "c3", 128, 128, True), ("u2", "up", 128, 64, True),
    ("c2a", "c3", 128, 64, True), ("c2b", "c3", 64, 64, True), ("u1", "up", 64, 32, True),
    ("c1a", "c3", 64, 32, True), ("c1b", "c3", 32, 32, True), ("head", "c1", 32, None, False),
]


NPARTS = 1024


class LossHandle:
    """Partial sums written by the masked-MSE kernel; value() copies them
    back and forms sum / (count * channels) on the host."""

    def __init__(self, parts, c):
        self.parts, self.c = parts, c

    def value(self) -> float:
        p = self.parts.cpu().numpy().astype(np.float64)
        n = p[-1] * self.c
        return float(p[:-1].sum() / n) if n > 0 else 0.0


def _ceil16(c):
    return (c + 15) // 16 * 16


def nn_lib():
    L = _mpm.lib()
    if not getattr(L, "_nn_ready", False):
        vp, i, ll, f = ct.c_void_p, ct.c_int, ct.c_longlong, ct.c_float
        L.mpm_nn_pack.argtypes = [vp, i, i, i, i, vp, vp]
        L.mpm_nn_conv.argtypes = [i, vp, i, i, i, i, i, i, i, vp, vp, i, vp, i, i, i, vp, i, vp]
        L.mpm_nn_wgrad.argtypes = [i, vp, i, i, i, i, i, i, i, vp, i, i, i, ll, vp, vp, i, vp]
        L.mpm_nn_bias_grad.argtypes = [vp, ll, i, i, i, vp, i, vp]
        L.mpm_nn_relu_bwd.argtypes = [vp, i, i, vp, i, i, ll, i, vp]
        L.mpm_nn_up_bwd.argtypes = [vp, i, i, vp, i, i, i, i, i, i, i, vp]
        L.mpm_nn_down_dgrad.argtypes = [vp, i, i, vp, i, i, vp, i, i, i, i, i, i, i, vp]
        L.mpm_nn_to_bf16.argtypes = [vp, i, ll, i, vp, i, i, i, vp]
        L.mpm_nn_masked_mse.argtypes = [vp, i, vp, vp, ll, i, vp, i, vp, i, vp]
        L.mpm_nn_adam.argtypes = [vp, vp, vp, vp, ll, f, f, f, f, i, vp]
        L.mpm_nn_bbox.argtypes = [vp, i, i, i, vp, vp]
        L.mpm_nn_crop_origin.argtypes = [vp, i, i, i, i, i, vp, vp]
        L.mpm_nn_crop.argtypes = [vp, i, i, i, vp, i, i, i, vp, i, vp]
        L._nn_ready = True
    return L


def _chk(r, what):
    if r != 0:
        raise RuntimeError(f"{what} failed ({r})")


class Act:
    """A BF16 channels-last activation buffer [n, d, h, w, c]."""

    def __init__(self, torch, n, d, h, w, c, device):
        self.n, self.d, self.h, self.w, self.c = n, d, h, w, c
        self.t = torch.zeros((n, d, h, w, c), dtype=torch.int16, device=device)

    @property
    def ptr(self):
        return self.t.data_ptr()

    @property
    def vox(self):
        return self.n * self.d * self.h * self.w


class UNet:
    """U-Net with FP32 master weights, trained by the library's kernels."""

    def __init__(self, cin: int = 8, cout: int = 4, width: int = 1, seed: int = 0, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = device
        self.cin, self.cout, self.width = cin, cout, width
        self.L = nn_lib()
        rng = np.random.default_rng(seed)
        self.layers = []
        self.params: Dict[str, "torch.Tensor"] = {}
        for name, kind, ci, co, relu in LAYERS:
            ci = _ceil16(cin) if ci is None else ci // width
            co = cout if co is None else co // width
            taps = TAPS[kind]
            fan_in = taps * (cin if name == "e1a" else ci)
            w = rng.normal(0.0, math.sqrt(2.0 / fan_in), (taps, ci, co))
            if name == "e1a":
                w[:, cin:, :] = 0.0            # padded input channels
            if name == "head":
                w *= 0.1                       # start near the zero update
            self.params[name + ".w"] = torch.tensor(w, dtype=torch.float32, device=device)
            self.params[name + ".b"] = torch.zeros(co, dtype=torch.float32, device=device)
            self.layers.append((name, kind, ci, co, relu))
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.step_t = 0
        self.packs = {}
        self.repack()
        self._bufs = None
        self._partial = None

    @property
    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    # ------------------------------------------------------------------ weights
    def repack(self):
        torch = self.torch
        for name, kind, ci, co, _ in self.layers:
            w = self.params[name + ".w"]
            taps = TAPS[kind]
            fw = torch.zeros(taps * _ceil16(ci) * _ceil16(co), dtype=torch.int16, device=self.device)
            if name == "e1a" and self.cin == 8:
                # the first layer sees the 8 real input channels (taps folded into the MFMA K)
                w8 = w[:, :8, :].contiguous()
                _chk(self.L.mpm_nn_pack(w8.data_ptr(), KIND[kind], 8, co, 0, fw.data_ptr(), self.stream), "pack")
            else:
                _chk(self.L.mpm_nn_pack(w.data_ptr(), KIND[kind], ci, co, 0, fw.data_ptr(), self.stream), "pack")
            bw = torch.zeros(taps * _ceil16(co) * _ceil16(ci), dtype=torch.int16, device=self.device)
            _chk(self.L.mpm_nn_pack(w.data_ptr(), KIND[kind], ci, co, 1, bw.data_ptr(), self.stream), "pack")
            self.packs[name] = (fw, bw)

    def export_weights(self) -> bytes:
        """The weight blob of mpm_surrogate_load (include/mpm.h): an int32
        header, then every layer's FP32 weights [taps][ci][co] and bias in
        network order."""
        hdr = np.array([0x554E504D, 1, self.cin, self.cout, self.width, len(self.layers), 0, 0], "<i4")
        parts = [hdr.tobytes()]
        for name, kind, ci, co, _ in self.layers:
            parts.append(np.ascontiguousarray(self.params[name + ".w"].detach().cpu().numpy(), "<f4").tobytes())
            parts.append(np.ascontiguousarray(self.params[name + ".b"].detach().cpu().numpy(), "<f4").tobytes())
        return b"".join(parts)

    def state_dict(self):
        return {k: v.detach().cpu().numpy() for k, v in self.params.items()}

    def load_state_dict(self, sd):
        for k, v in sd.items():
            self.params[k].copy_(self.torch.tensor(np.asarray(v), dtype=self.torch.float32))
        self.repack()

    # ------------------------------------------------------------------ buffers
    def _alloc(self, n, shape):
        key = (n,) + tuple(shape)
        if self._bufs is not None and self._bufs["key"] == key:
            return self._bufs
        torch, dev, w = self.torch, self.device, self.width
        c1, c2, c3 = 32 // w, 64 // w, 128 // w
        L1 = tuple(shape)
        L2 = tuple(d // 2 for d in shape)
        L3 = tuple(d // 4 for d in shape)
        A = lambda lv, c: Act(torch, n, lv[0], lv[1], lv[2], c, dev)
        b = {"key": key}
        b["x"] = A(L1, _ceil16(self.cin))
        b["a1"], b["cat1"], b["a2"], b["a3"] = A(L1, c1), A(L1, 2 * c1), A(L2, c2), A(L2, c2)
        b["cat2"], b["a4"], b["a5"], b["a6"] = A(L2, 2 * c2), A(L3, c3), A(L3, c3), A(L3, c3)
        b["a7"], b["a8"], b["a9"], b["a10"] = A(L2, c2), A(L2, c2), A(L1, c1), A(L1, c1)
        b["pred"] = torch.zeros((n,) + L1 + (self.cout,), dtype=torch.float32, device=dev)
        # gradients
        b["gpred"] = A(L1, 16)
        b["g10"], b["g9"], b["gcat1"], b["gf1"] = A(L1, c1), A(L1, c1), A(L1, 2 * c1), A(L1, c2)
        b["g8"], b["g7"], b["gcat2"], b["gf2"] = A(L2, c2), A(L2, c2), A(L2, 2 * c2), A(L2, c3)
        b["g6"], b["g5"], b["g4"], b["g3"], b["g2"], b["g1"] = (A(L3, c3), A(L3, c3), A(L3, c3), A(L2, c2),
                                                               A(L2, c2), A(L1, c1))
        self._bufs = b
        return b

    # ------------------------------------------------------------------ forward
    def _conv(self, name, x: Act, x_off, cin, y: Optional[Act], y_off, y32=None, cy32=0):
        _, kind, ci, co, relu = [l for l in self.layers if l[0] == name][0]
        fw = self.packs[name][0]
        r = self.L.mpm_nn_conv(KIND[kind], x.ptr, x.n, x.d, x.h, x.w, x.c, x_off, cin, fw.data_ptr(),
                               self.params[name + ".b"].data_ptr(), int(relu), y.ptr if y else None,
                               y.c if y else 0, y_off, co, y32.data_ptr() if y32 is not None else None, cy32,
                               self.stream)
        _chk(r, "conv " + name)

    def forward(self, x32, out=None):
        """x32: FP32 tensor [n, D, H, W, >= cin channels] on the device (D, H, W
        multiples of 4) -> FP32 [n, D, H, W, cout] (written into `out` when
        given, a contiguous tensor)."""
        n, shape = x32.shape[0], tuple(x32.shape[1:4])
        assert all(d % 4 == 0 for d in shape) and x32.is_contiguous() and x32.shape[-1] >= self.cin
        nvox = n * shape[0] * shape[1] * shape[2]
        b = self._alloc(n, shape)
        pred = b["pred"]
        if out is not None:
            assert out.is_contiguous() and tuple(out.shape) == (n,) + shape + (self.cout,)
            pred = out
        w = self.width
        c1, c2, c3 = 32 // w, 64 // w, 128 // w
        _chk(self.L.mpm_nn_to_bf16(x32.data_ptr(), x32.shape[-1], nvox, self.cin, b["x"].ptr, b["x"].c, 0,
                                   b["x"].c, self.stream), "to_bf16")
        self._conv("e1a", b["x"], 0, 8 if self.cin == 8 else b["x"].c, b["a1"], 0)
        self._conv("e1b", b["a1"], 0, c1, b["cat1"], c1)
        self._conv("d1", b["cat1"], c1, c1, b["a2"], 0)
        self._conv("e2a", b["a2"], 0, c2, b["a3"], 0)
        self._conv("e2b", b["a3"], 0, c2, b["cat2"], c2)
        self._conv("d2", b["cat2"], c2, c2, b["a4"], 0)
        self._conv("e3a", b["a4"], 0, c3, b["a5"], 0)
        self._conv("e3b", b["a5"], 0, c3, b["a6"], 0)
        self._conv("u2", b["a6"], 0, c3, b["cat2"], 0)
        self._conv("c2a", b["cat2"], 0, 2 * c2, b["a7"], 0)
        self._conv("c2b", b["a7"], 0, c2, b["a8"], 0)
        self._conv("u1", b["a8"], 0, c2, b["cat1"], 0)
        self._conv("c1a", b["cat1"], 0, 2 * c1, b["a9"], 0)
        self._conv("c1b", b["a9"], 0, c1, b["a10"], 0)
        self._conv("head", b["a10"], 0, c1, None, 0, pred, self.cout)
        return pred

    # ------------------------------------------------------------------ backward
    def _wgrad(self, name, x: Act, x_off, cin, g: Act, g_off):
        _, kind, ci, co, _ = [l for l in self.layers if l[0] == name][0]
        torch = self.torch
        # output voxels of this layer
        if kind == "up":
            vox = x.n * 8 * x.d * x.h * x.w
        elif kind == "down":
            vox = x.n * x.d * x.h * x.w // 8
        else:
            vox = x.vox
        # voxels per partial sum: about 256 partials per layer, so that even a small batch gives the
        # weight-gradient kernel enough workgroups (its grid is partials x input-channel groups x 4)
        chunk = min(8192, max(256, (vox // 256 + 15) // 16 * 16))
        nchunk = (vox + chunk - 1) // chunk
        need = nchunk * TAPS[kind] * cin * co
        if self._partial is None or self._partial.numel() < need:
            self._partial = torch.zeros(need, dtype=torch.float32, device=self.device)
        r = self.L.mpm_nn_wgrad(KIND[kind], x.ptr, x.n, x.d, x.h, x.w, x.c, x_off, cin, g.ptr, g.c, g_off, co,
                                chunk, self._partial.data_ptr(), self.grads[name + ".w"].data_ptr(), 0, self.stream)
        _chk(r, "wgrad " + name)
        _chk(self.L.mpm_nn_bias_grad(g.ptr, vox, g.c, g_off, co, self.grads[name + ".b"].data_ptr(), 0, self.stream),
             "bias grad " + name)

    def _dgrad(self, name, g: Act, g_off, gx: Act, gx_off):
        """gx[slice] = adjoint conv of g (3^3 / 1^3 kinds, same resolution)."""
        _, kind, ci, co, _ = [l for l in self.layers if l[0] == name][0]
        bw = self.packs[name][1]
        k = KIND["c1"] if kind == "c1" else KIND["c3"]
        r = self.L.mpm_nn_conv(k, g.ptr, g.n, g.d, g.h, g.w, g.c, g_off, _ceil16(co), bw.data_ptr(), None, 0,
                               gx.ptr, gx.c, gx_off, ci, None, 0, self.stream)
        _chk(r, "dgrad " + name)

    def _relu_bwd(self, g: Act, g_off, y: Act, y_off, c):
        _chk(self.L.mpm_nn_relu_bwd(g.ptr, g.c, g_off, y.ptr, y.c, y_off, g.vox, c, self.stream), "relu_bwd")

    def backward(self, gpred: Act):
        """gpred: BF16 gradient of the output (16 channels, cout used)."""
        b = self._bufs
        w = self.width
        c1, c2, c3 = 32 // w, 64 // w, 128 // w
        L, s = self.L, self.stream
        # head
        self._wgrad("head", b["a10"], 0, c1, gpred, 0)
        self._dgrad("head", gpred, 0, b["g10"], 0)
        # c1b, c1a
        self._relu_bwd(b["g10"], 0, b["a10"], 0, c1)
        self._wgrad("c1b", b["a9"], 0, c1, b["g10"], 0)
        self._dgrad("c1b", b["g10"], 0, b["g9"], 0)
        self._relu_bwd(b["g9"], 0, b["a9"], 0, c1)
        self._wgrad("c1a", b["cat1"], 0, 2 * c1, b["g9"], 0)
        self._dgrad("c1a", b["g9"], 0, b["gcat1"], 0)
        # u1: gradient of the upsampled conv, then sum the children
        self._relu_bwd(b["gcat1"], 0, b["cat1"], 0, c1)
        self._wgrad("u1", b["a8"], 0, c2, b["gcat1"], 0)
        self._dgrad("u1", b["gcat1"], 0, b["gf1"], 0)
        a8 = b["a8"]
        _chk(L.mpm_nn_up_bwd(b["gf1"].ptr, b["gf1"].c, 0, b["g8"].ptr, b["g8"].c, 0, a8.n, a8.d, a8.h, a8.w, c2, s),
             "up_bwd")
        # c2b, c2a
        self._relu_bwd(b["g8"], 0, b["a8"], 0, c2)
        self._wgrad("c2b", b["a7"], 0, c2, b["g8"], 0)
        self._dgrad("c2b", b["g8"], 0, b["g7"], 0)
        self._relu_bwd(b["g7"], 0, b["a7"], 0, c2)
        self._wgrad("c2a", b["cat2"], 0, 2 * c2, b["g7"], 0)
        self._dgrad("c2a", b["g7"], 0, b["gcat2"], 0)
        # u2
        self._relu_bwd(b["gcat2"], 0, b["cat2"], 0, c2)
        self._wgrad("u2", b["a6"], 0, c3, b["gcat2"], 0)
        self._dgrad("u2", b["gcat2"], 0, b["gf2"], 0)
        a6 = b["a6"]
        _chk(L.mpm_nn_up_bwd(b["gf2"].ptr, b["gf2"].c, 0, b["g6"].ptr, b["g6"].c, 0, a6.n, a6.d, a6.h, a6.w, c3, s),
             "up_bwd")
        # e3b, e3a
        self._relu_bwd(b["g6"], 0, b["a6"], 0, c3)
        self._wgrad("e3b", b["a5"], 0, c3, b["g6"], 0)
        self._dgrad("e3b", b["g6"], 0, b["g5"], 0)
        self._relu_bwd(b["g5"], 0, b["a5"], 0, c3)
        self._wgrad("e3a", b["a4"], 0, c3, b["g5"], 0)
        self._dgrad("e3a", b["g5"], 0, b["g4"], 0)
        # d2: input was cat2[c2:]; its gradient adds to the skip gradient there
        self._relu_bwd(b["g4"], 0, b["a4"], 0, c3)
        self._wgrad("d2", b["cat2"], c2, c2, b["g4"], 0)
        cat2 = b["cat2"]
        _chk(L.mpm_nn_down_dgrad(b["g4"].ptr, b["g4"].c, 0, self.params["d2.w"].data_ptr(), c2, c3, b["gcat2"].ptr,
                                 b["gcat2"].c, c2, cat2.n, cat2.d, cat2.h, cat2.w, 1, s), "down_dgrad")
        # e2b, e2a
        self._relu_bwd(b["gcat2"], c2, b["cat2"], c2, c2)
        self._wgrad("e2b", b["a3"], 0, c2, b["gcat2"], c2)
        self._dgrad("e2b", b["gcat2"], c2, b["g3"], 0)
        self._relu_bwd(b["g3"], 0, b["a3"], 0, c2)
        self._wgrad("e2a", b["a2"], 0, c2, b["g3"], 0)
        self._dgrad("e2a", b["g3"], 0, b["g2"], 0)
        # d1
        self._relu_bwd(b["g2"], 0, b["a2"], 0, c2)
        self._wgrad("d1", b["cat1"], c1, c1, b["g2"], 0)
        cat1 = b["cat1"]
        _chk(L.mpm_nn_down_dgrad(b["g2"].ptr, b["g2"].c, 0, self.params["d1.w"].data_ptr(), c1, c2, b["gcat1"].ptr,
                                 b["gcat1"].c, c1, cat1.n, cat1.d, cat1.h, cat1.w, 1, s), "down_dgrad")
        # e1b, e1a
        self._relu_bwd(b["gcat1"], c1, b["cat1"], c1, c1)
        self._wgrad("e1b", b["a1"], 0, c1, b["gcat1"], c1)
        self._dgrad("e1b", b["gcat1"], c1, b["g1"], 0)
        self._relu_bwd(b["g1"], 0, b["a1"], 0, c1)
        self._wgrad("e1a", b["x"], 0, b["x"].c, b["g1"], 0)
        return self.grads

    # ------------------------------------------------------------------ training
    def loss_and_grad(self, pred, target, mask):
        """Masked MSE on the device; writes the output gradient buffer.
        Returns (loss handle, gradient); the handle's value() reads it back."""
        b = self._bufs
        n_vox = pred.shape[0] * pred.shape[1] * pred.shape[2] * pred.shape[3]
        parts = self.torch.zeros(NPARTS + 1, dtype=self.torch.float32, device=self.device)
        _chk(self.L.mpm_nn_masked_mse(pred.data_ptr(), pred.shape[-1], target.data_ptr(), mask.data_ptr(), n_vox,
                                      self.cout, b["gpred"].ptr, b["gpred"].c, parts.data_ptr(), NPARTS,
                                      self.stream), "masked_mse")
        return LossHandle(parts, self.cout), b["gpred"]

    def adam(self, lr=3e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.step_t += 1
        for k, p in self.params.items():
            _chk(self.L.mpm_nn_adam(p.data_ptr(), self.grads[k].data_ptr(), self.adam_m[k].data_ptr(),
                                    self.adam_v[k].data_ptr(), p.numel(), lr, b1, b2, eps, self.step_t, self.stream),
                 "adam")
        self.repack()

    def train_step(self, x, target, mask, lr=3e-4):
        pred = self.forward(x)
        loss, g = self.loss_and_grad(pred, target, mask)
        self.backward(g)
        self.adam(lr)
        return loss
