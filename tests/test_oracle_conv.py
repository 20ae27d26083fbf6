"""Pins for the oracle's convolution network: a brute-force loop over every
output voxel and tap, central finite differences of the backward pass, the
translation equivariance of circular padding along x and y, and Adam's
first step (whose bias correction makes it lr * sign(g) up to eps)."""
import numpy as np
import pytest

from oracle import conv as Cv


def _brute(x, W, b, dil):
    co, ci = W.shape[:2]
    _, nz, ny, nx = x.shape
    y = np.zeros((co, nz, ny, nx))
    for o in range(co):
        for z in range(nz):
            for yy in range(ny):
                for xx in range(nx):
                    s = b[o]
                    for c in range(ci):
                        for dz in range(3):
                            zz = z + (dz - 1) * dil
                            if zz < 0 or zz >= nz:
                                continue
                            for dy in range(3):
                                for dx in range(3):
                                    s += W[o, c, dz, dy, dx] * x[c, zz, (yy + (dy - 1) * dil) % ny,
                                                                   (xx + (dx - 1) * dil) % nx]
                    y[o, z, yy, xx] = s
    return y


@pytest.mark.parametrize("dil", [1, 2, 4])
def test_conv_matches_brute_force(dil):
    rng = np.random.default_rng(dil)
    x = rng.standard_normal((2, 7, 5, 6))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.abs(Cv.conv3d(x, W, b, dil) - _brute(x, W, b, dil)).max() < 1e-12


@pytest.mark.parametrize("dil,cin,weighted", [((1, 2, 4, 1), 1, False), ((1, 2, 4, 8, 2, 1), 4, True),
                                              ((2, 1), 1, True)])
def test_backward_finite_differences(dil, cin, weighted):
    rng = np.random.default_rng(len(dil))
    params = Cv.init_params(rng, channels=4, in_channels=cin, n_layers=len(dil))
    for W, b in params:
        b += rng.standard_normal(b.shape) * 0.1
    x = rng.standard_normal((cin, 9, 6, 6))
    t = rng.standard_normal((1, 9, 6, 6))
    w = rng.uniform(0.5, 3.0, (1, 9, 6, 6)) if weighted else None

    def loss_of():
        return Cv.mse(Cv.forward(x, params, dilations=dil)[0], t, w)[0]

    out, cache = Cv.forward(x, params, dilations=dil)
    loss, dout = Cv.mse(out, t, w)
    grads = Cv.backward(params, cache, dout)
    eps = 1e-6
    for li in range(len(dil)):
        W, b = params[li]
        for idx in [(0, 0, 1, 1, 1), (min(1, W.shape[0] - 1), W.shape[1] - 1, 0, 2, 1), (0, 0, 2, 0, 2)]:
            old = W[idx]
            W[idx] = old + eps
            lp = loss_of()
            W[idx] = old - eps
            lm = loss_of()
            W[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)
        old = b[0]
        b[0] = old + eps
        lp = loss_of()
        b[0] = old - eps
        lm = loss_of()
        b[0] = old
        assert grads[li][1][0] == pytest.approx((lp - lm) / (2 * eps), rel=1e-6, abs=1e-10)


def test_weighted_mse_closed_forms():
    rng = np.random.default_rng(5)
    p, t = rng.standard_normal((1, 4, 3, 3)), rng.standard_normal((1, 4, 3, 3))
    assert Cv.mse(p, t, np.ones_like(p))[0] == pytest.approx(Cv.mse(p, t)[0], rel=1e-15)
    m = np.zeros_like(p)
    m[0, 1] = 1.0
    d = (p - t)[0, 1]
    assert Cv.mse(p, t, m)[0] == pytest.approx(np.sum(d * d) / p.size, rel=1e-14)


def test_translation_equivariance_xy():
    rng = np.random.default_rng(3)
    params = Cv.init_params(rng, channels=4)
    x = rng.standard_normal((1, 8, 6, 6))
    y, _ = Cv.forward(x, params)
    ys, _ = Cv.forward(np.roll(x, (2, -1), axis=(2, 3)), params)
    assert np.abs(np.roll(y, (2, -1), axis=(2, 3)) - ys).max() < 1e-12


def test_adam_first_step_and_quadratic():
    w, m, v = np.array([1.0, -2.0]), np.zeros(2), np.zeros(2)
    g = np.array([0.3, -5.0])
    w1, m1, v1 = Cv.adam_step(w, g, m, v, 1, lr=1e-2)
    assert np.allclose(w1, w - 1e-2 * np.sign(g), atol=1e-9)
    # minimises a quadratic
    w = np.array([3.0])
    m = v = np.zeros(1)
    for t in range(1, 3001):
        w, m, v = Cv.adam_step(w, 2 * (w - 0.5), m, v, t, lr=1e-2)
    assert abs(w[0] - 0.5) < 1e-3
