"""Pins of the FP64 U-Net oracle (no GPU): brute-force convolution, adjoint
identities, finite differences through the whole network, Adam's first step."""
import numpy as np
import pytest

from oracle import unet


def _conv_brute(x, w, b, stride=1, pad=1):
    """Direct 7-loop convolution written from its definition."""
    n, d, h, wd, ci = x.shape
    k = w.shape[0]
    co = w.shape[-1]
    od, oh, ow = (d + 2 * pad - k) // stride + 1, (h + 2 * pad - k) // stride + 1, (wd + 2 * pad - k) // stride + 1
    y = np.zeros((n, od, oh, ow, co))
    for s in range(n):
        for i in range(od):
            for j in range(oh):
                for l in range(ow):
                    acc = b.copy()
                    for a in range(k):
                        for c in range(k):
                            for e in range(k):
                                ii, jj, ll = i * stride + a - pad, j * stride + c - pad, l * stride + e - pad
                                if 0 <= ii < d and 0 <= jj < h and 0 <= ll < wd:
                                    acc += x[s, ii, jj, ll] @ w[a, c, e]
                    y[s, i, j, l] = acc
    return y


def test_conv3_and_down_match_brute_force():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 6, 3))
    w = rng.normal(size=(3, 3, 3, 3, 4))
    b = rng.normal(size=4)
    assert np.allclose(unet.conv3(x, w, b), _conv_brute(x, w, b), atol=1e-12)
    w2 = rng.normal(size=(2, 2, 2, 3, 5))
    x2 = rng.normal(size=(1, 4, 4, 6, 3))
    assert np.allclose(unet.down(x2, w2, b[:1].repeat(5)), _conv_brute(x2, w2, b[:1].repeat(5), stride=2, pad=0),
                       atol=1e-12)


@pytest.mark.parametrize("kind", ["c3", "down", "up", "c1"])
def test_adjoint_identities(kind):
    """<y, L x> = <L^T y, x> for each linear layer (bias zero)."""
    rng = np.random.default_rng(1)
    k = unet.KSIZE[kind]
    w = rng.normal(size=(k, k, k, 3, 4))
    b = np.zeros(4)
    x = rng.normal(size=(2, 4, 4, 4, 3))
    if kind == "c3":
        y = unet.conv3(x, w, b)
        g = rng.normal(size=y.shape)
        gx = unet.conv3_backward(x, w, g)[0]
    elif kind == "down":
        y = unet.down(x, w, b)
        g = rng.normal(size=y.shape)
        gx = unet.down_backward(x, w, g)[0]
    elif kind == "up":
        y = unet.conv3(unet.upsample(x), w, b)
        g = rng.normal(size=y.shape)
        gx = unet.upsample_backward(unet.conv3_backward(unet.upsample(x), w, g)[0])
    else:
        y = unet.conv1(x, w, b)
        g = rng.normal(size=y.shape)
        gx = unet.conv1_backward(x, w, g)[0]
    assert abs((g * y).sum() - (gx * x).sum()) < 1e-10 * max(1.0, abs((g * y).sum()))


def test_network_gradients_by_finite_differences():
    rng = np.random.default_rng(2)
    cin, cout, width = 3, 2, 8          # hidden channels 4 / 8 / 16 on an 8^3 grid
    params = unet.init_params(cin, cout, seed=3, width=width)
    for k in params:
        if k.endswith(".b"):
            params[k] = 0.1 * rng.normal(size=params[k].shape)
    x = rng.normal(size=(1, 8, 8, 8, cin))
    target = rng.normal(size=(1, 8, 8, 8, cout))
    mask = (rng.random((1, 8, 8, 8)) < 0.6).astype(float)

    def loss_of(p):
        y, _ = unet.forward(p, x, cin, cout, width)
        return unet.masked_mse(y, target, mask)[0]

    y, cache = unet.forward(params, x, cin, cout, width)
    loss, gy = unet.masked_mse(y, target, mask)
    grads = unet.backward(params, cache, gy, cin, cout, width)
    checked = 0
    for k in sorted(params):
        flat = params[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            h = 1e-5 * max(1.0, abs(old))
            flat[idx] = old + h
            lp = loss_of(params)
            flat[idx] = old - h
            lm = loss_of(params)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)
            checked += 1
    assert checked > 40


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 0.0])}
    st = {}
    unet.adam_step(p, g, st, lr=1e-2)
    assert np.allclose(p["w"], [1.0 - 1e-2, -2.0 + 1e-2, 3.0], atol=1e-7)


def test_bf16_round_values():
    vals = np.array([1.0, 1.00390625, 1.001953125, 3.14159265, -2.5e-3, 65504.0])
    r = unet.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0           # 1 + 2^-8 is a tie: even mantissa
    assert r[2] == 1.0                      # ties to even at 1 + 2^-9
    assert abs(r[3] - 3.140625) < 1e-12
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8)
