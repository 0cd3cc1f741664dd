"""FP64 NumPy oracle of the grid U-Net surrogate -- TEST INFRASTRUCTURE ONLY.

Plain, slow reference for the surrogate network's forward pass, backward
pass, masked MSE loss and Adam update.  Only the tests and the smoke check
use it; the product path runs its own HIP kernels.

The paper has no learned component; the network shape is the reading
taken here of the grid surrogate (a 3-level grid U-Net, 32/64/128 channels,
3^3 convolutions, predicting the grid velocity / mass change of a
25-substep block from mass, momentum and collider fields):

  enc1: conv3(Cin->32)+ReLU, conv3(32->32)+ReLU            at R^3
  down1: conv2 stride 2 (32->64)+ReLU                       -> (R/2)^3
  enc2: conv3(64->64)+ReLU x2
  down2: conv2 stride 2 (64->128)+ReLU                      -> (R/4)^3
  enc3: conv3(128->128)+ReLU x2
  up2: nearest x2, conv3(128->64)+ReLU, concat enc2         -> 128 ch
  dec2: conv3(128->64)+ReLU, conv3(64->64)+ReLU
  up1: nearest x2, conv3(64->32)+ReLU, concat enc1          -> 64 ch
  dec1: conv3(64->32)+ReLU, conv3(32->32)+ReLU
  head: conv1(32->Cout)

Tensors are channels-last [N, D, H, W, C]; convolution weights are
[kd, kh, kw, Cin, Cout]; 3^3 convolutions use zero padding 1; the stride-2
convolution reads the 2^3 children of each coarse voxel.  Every convolution
is written as the sum over kernel taps of shifted views times the tap's
weight matrix (a plain matmul per tap).
"""
from __future__ import annotations

import numpy as np

LAYERS = [
    # name, kind, cin, cout, relu
    ("e1a", "c3", None, 32, True),
    ("e1b", "c3", 32, 32, True),
    ("d1", "down", 32, 64, True),
    ("e2a", "c3", 64, 64, True),
    ("e2b", "c3", 64, 64, True),
    ("d2", "down", 64, 128, True),
    ("e3a", "c3", 128, 128, True),
    ("e3b", "c3", 128, 128, True),
    ("u2", "up", 128, 64, True),
    ("c2a", "c3", 128, 64, True),
    ("c2b", "c3", 64, 64, True),
    ("u1", "up", 64, 32, True),
    ("c1a", "c3", 64, 32, True),
    ("c1b", "c3", 32, 32, True),
    ("head", "c1", 32, None, False),
]

KSIZE = {"c3": 3, "up": 3, "down": 2, "c1": 1}


def layer_shapes(cin: int, cout: int, width: int = 1):
    """[(name, kind, cin, cout, relu)] with the model's in / out channels
    filled in; `width` divides the hidden channel counts (small test nets)."""
    out = []
    for name, kind, ci, co, relu in LAYERS:
        ci = cin if ci is None else ci // width
        co = cout if co is None else co // width
        out.append((name, kind, ci, co, relu))
    return out


def init_params(cin, cout, seed=0, width=1):
    rng = np.random.default_rng(seed)
    params = {}
    for name, kind, ci, co, _ in layer_shapes(cin, cout, width):
        k = KSIZE[kind]
        fan_in = k ** 3 * ci
        params[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / fan_in), (k, k, k, ci, co))
        params[name + ".b"] = np.zeros(co)
    return params


# ---------------------------------------------------------------- primitives
def conv3(x, w, b):
    """3^3 convolution, zero padding 1: y[v] = b + sum_t x[v + t - 1] @ w[t]."""
    n, d, h, wd, ci = x.shape
    xp = np.zeros((n, d + 2, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((n, d, h, wd, w.shape[-1])) + b
    for a in range(3):
        for c in range(3):
            for e in range(3):
                y += xp[:, a:a + d, c:c + h, e:e + wd] @ w[a, c, e]
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 w.r.t. its input, weights and bias."""
    n, d, h, wd, ci = x.shape
    xp = np.zeros((n, d + 2, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            for e in range(3):
                view = xp[:, a:a + d, c:c + h, e:e + wd]
                gw[a, c, e] = view.reshape(-1, ci).T @ gy.reshape(-1, gy.shape[-1])
                gxp[:, a:a + d, c:c + h, e:e + wd] += gy @ w[a, c, e].T
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gy.reshape(-1, gy.shape[-1]).sum(0)


def down(x, w, b):
    """2^3 stride-2 convolution: y[V] = b + sum_t x[2V + t] @ w[t]."""
    y = b + np.zeros(x.shape[:1] + tuple(s // 2 for s in x.shape[1:4]) + (w.shape[-1],))
    for a in range(2):
        for c in range(2):
            for e in range(2):
                y += x[:, a::2, c::2, e::2] @ w[a, c, e]
    return y


def down_backward(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    ci = x.shape[-1]
    for a in range(2):
        for c in range(2):
            for e in range(2):
                view = x[:, a::2, c::2, e::2]
                gw[a, c, e] = view.reshape(-1, ci).T @ gy.reshape(-1, gy.shape[-1])
                gx[:, a::2, c::2, e::2] += gy @ w[a, c, e].T
    return gx, gw, gy.reshape(-1, gy.shape[-1]).sum(0)


def upsample(x):
    """Nearest-neighbour x2 in every spatial axis."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def upsample_backward(g):
    n, d, h, w, c = g.shape
    return g.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def conv1(x, w, b):
    return x @ w[0, 0, 0] + b


def conv1_backward(x, w, gy):
    ci = x.shape[-1]
    gw = np.zeros_like(w)
    gw[0, 0, 0] = x.reshape(-1, ci).T @ gy.reshape(-1, gy.shape[-1])
    return gy @ w[0, 0, 0].T, gw, gy.reshape(-1, gy.shape[-1]).sum(0)


# ---------------------------------------------------------------- network
def forward(params, x, cin, cout, width=1, q=None):
    """Returns the output and a cache of every layer input / pre-activation.

    q (optional) is a rounding function applied where a BF16 implementation
    stores values: the network input, every weight tensor fed to a
    convolution and every hidden activation (the head output stays exact).
    q = None is the exact network."""
    q_ = q if q is not None else (lambda a: a)
    cache = {}
    skips = {}
    h = q_(x)
    for name, kind, ci, co, relu in layer_shapes(cin, cout, width):
        if name == "c2a":
            h = np.concatenate([h, skips["e2b"]], axis=-1)
        if name == "c1a":
            h = np.concatenate([h, skips["e1b"]], axis=-1)
        w, b = q_(params[name + ".w"]), params[name + ".b"]
        inp = upsample(h) if kind == "up" else h
        cache[name] = inp
        if kind in ("c3", "up"):
            z = conv3(inp, w, b)
        elif kind == "down":
            z = down(inp, w, b)
        else:
            z = conv1(inp, w, b)
        cache[name + ".z"] = z
        h = q_(np.maximum(z, 0.0)) if relu else z
        if name in ("e1b", "e2b"):
            skips[name] = h
    return h, cache


def backward(params, cache, gout, cin, cout, width=1, q=None):
    """Gradients of every parameter for the output gradient `gout`.

    With q (see forward): every convolution adjoint is computed with the
    rounded weights, and every input gradient is rounded where a BF16
    implementation stores it -- after each convolution adjoint, after the
    upsampling adjoint, and where a skip gradient is summed in (the
    stride-2 adjoint writes straight into that sum and is rounded only
    there).  Parameter gradients stay exact."""
    q_ = q if q is not None else (lambda a: a)
    grads = {}
    shapes = layer_shapes(cin, cout, width)
    g = gout
    gskip = {}
    for name, kind, ci, co, relu in reversed(shapes):
        if name in gskip:
            g = q_(g + gskip.pop(name))
        z = cache[name + ".z"]
        if relu:
            g = g * (z > 0)
        w = params[name + ".w"]
        inp = cache[name]
        if kind in ("c3", "up"):
            gin, gw, gb = conv3_backward(inp, q_(w), g)
            gin = q_(gin)
        elif kind == "down":
            gin, gw, gb = down_backward(inp, q_(w), g)
        else:
            gin, gw, gb = conv1_backward(inp, q_(w), g)
            gin = q_(gin)
        grads[name + ".w"], grads[name + ".b"] = gw, gb
        if kind == "up":
            gin = q_(upsample_backward(gin))
        if name == "c1a":
            # split the gradient of concat([up1 output, e1b output])
            n_up = [s for s in shapes if s[0] == "u1"][0][3]
            gskip["e1b"] = gin[..., n_up:]
            gin = gin[..., :n_up]
        if name == "c2a":
            n_up = [s for s in shapes if s[0] == "u2"][0][3]
            gskip["e2b"] = gin[..., n_up:]
            gin = gin[..., :n_up]
        g = gin
    return grads


def masked_mse(pred, target, mask):
    """mean over masked voxels and channels of (pred - target)^2, and its gradient."""
    n = max(float(mask.sum()) * pred.shape[-1], 1.0)
    diff = (pred - target) * mask[..., None]
    return float((diff ** 2).sum() / n), 2.0 * diff / n


def adam_step(params, grads, state, lr=3e-4, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; `state` holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m." + k, np.zeros_like(params[k]))
        v = state.setdefault("v." + k, np.zeros_like(params[k]))
        m *= b1
        m += (1 - b1) * grads[k]
        v *= b2
        v += (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
