"""Oracle: the 3-D convolutional surrogate of the initial potential.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's self-consistent loop starts from some potential and iterates
(Sec. III-A); the surrogate proposes that start from the donor map.  The
network is fixed here by its definition: L 3x3x3 convolutions
c_in -> C -> ... -> C -> 1, one dilation per layer (default four layers with
dilations (1, 2, 4, 1)), ReLU after all but the last, circular padding along
x and y (the slab is periodic there) and zero padding along z.  Tensors are [channels, nz, ny, nx]; weights [c_out, c_in, 3, 3, 3]
indexed [dz][dy][dx] with tap offset (d - 1) * dilation.

forward() optionally rounds every layer's output to FP16 (half_acts=True)
and backward() every upstream gradient (half_grads=True), the storage
precision of activations and gradients on the device; arithmetic is FP64.
"""
from __future__ import annotations

import numpy as np

DILATIONS = (1, 2, 4, 1)


def shifted(x, oz, oy, ox):
    """s[c, z, y, x] = x[c, z + oz, (y + oy) % ny, (x + ox) % nx], zero when
    z + oz is outside [0, nz)."""
    s = np.roll(x, shift=(-oy, -ox), axis=(2, 3))
    out = np.zeros_like(s)
    nz = x.shape[1]
    if oz >= 0:
        out[:, : nz - oz] = s[:, oz:]
    else:
        out[:, -oz:] = s[:, : nz + oz]
    return out


def conv3d(x, W, b, dil):
    """y[o] = b[o] + sum_{c, taps} W[o, c, t] * x[c] shifted by the tap."""
    y = np.zeros((W.shape[0],) + x.shape[1:]) + b[:, None, None, None]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                xs = shifted(x, (dz - 1) * dil, (dy - 1) * dil, (dx - 1) * dil)
                y += np.einsum("oc,czyx->ozyx", W[:, :, dz, dy, dx], xs)
    return y


def conv3d_backward(x, W, dil, dy):
    """Gradients of sum(dy * conv3d(x, W, b)) w.r.t. x, W and b."""
    dx = np.zeros_like(x, dtype=np.float64)
    dW = np.zeros_like(W, dtype=np.float64)
    for dz in range(3):
        for dyy in range(3):
            for dxx in range(3):
                oz, oy, ox = (dz - 1) * dil, (dyy - 1) * dil, (dxx - 1) * dil
                xs = shifted(x, oz, oy, ox)
                dW[:, :, dz, dyy, dxx] = np.einsum("ozyx,czyx->oc", dy, xs)
                # adjoint of the shift: shift back by the opposite offset
                dx += shifted(np.einsum("oc,ozyx->czyx", W[:, :, dz, dyy, dxx], dy), -oz, -oy, -ox)
    db = dy.sum(axis=(1, 2, 3))
    return dx, dW, db


def init_params(rng, channels=32, scale=None, in_channels=1, n_layers=4):
    """He-style random init of the layers (FP32-representable)."""
    shapes = [(channels, in_channels)] + [(channels, channels)] * (n_layers - 2) + [(1, channels)]
    params = []
    for co, ci in shapes:
        std = np.sqrt(2.0 / (27 * ci)) if scale is None else scale
        W = (rng.standard_normal((co, ci, 3, 3, 3)) * std).astype(np.float32).astype(np.float64)
        b = np.zeros(co)
        params.append((W, b))
    return params


def _half(a):
    return a.astype(np.float16).astype(np.float64)


def forward(x, params, half_acts=False, half_weights=False, dilations=DILATIONS):
    """Network output [1, nz, ny, nx] and the cache for backward."""
    assert len(dilations) == len(params)
    last = len(params) - 1
    acts = [x]
    pres = []
    h = x
    for li, ((W, b), dil) in enumerate(zip(params, dilations)):
        Wl = _half(W) if half_weights else W
        bl = _half(b) if half_weights else b
        pre = conv3d(h, Wl, bl, dil)
        pres.append(pre)
        h = np.maximum(pre, 0.0) if li < last else pre
        if half_acts and li < last:
            h = _half(h)
        acts.append(h)
    return h, dict(acts=acts, pres=pres, dilations=tuple(dilations))


def backward(params, cache, dout, half_weights=False, half_grads=False):
    """Gradients [(dW, db)] for dout = d loss / d output.  half_grads rounds
    the upstream gradient of every layer to FP16 (after the ReLU mask), the
    precision the device stores it in; arithmetic stays FP64."""
    dil = cache["dilations"]
    last = len(params) - 1
    grads = [None] * len(params)
    g = _half(dout) if half_grads else dout
    for li in range(last, -1, -1):
        W, b = params[li]
        Wl = _half(W) if half_weights else W
        if li < last:
            g = g * (cache["pres"][li] > 0)
            if half_grads:
                g = _half(g)
        dx, dW, db = conv3d_backward(cache["acts"][li], Wl, dil[li], g)
        grads[li] = (dW, db)
        g = dx
    return grads


def mse(pred, target, weight=None):
    """mean(w (pred - target)^2) (w = 1 when weight is None) and its gradient."""
    d = pred - target
    w = np.ones_like(d) if weight is None else np.broadcast_to(weight, d.shape)
    return float(np.mean(w * d * d)), 2.0 * w * d / d.size


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), t counted from 1.  Returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
