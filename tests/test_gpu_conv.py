"""GPU parity of the surrogate's kernels against the oracle network.

The GPU keeps activations and weights in FP16 with FP32 accumulation; the
oracle computes in FP64 on the same FP16-rounded weights, rounding each
hidden layer's output and each upstream gradient to FP16 like the GPU
stores them.  Bars: forward and gradients 1e-3 normwise per layer on random
weights (a few FP16 rounding boundaries fall differently under FP32 vs FP64
accumulation; through more layers those differences compound, so deeper
nets and the weighted loss are checked instead on exactly representable
weights and data, where the bar is 1e-6); Adam's first step is
-lr * sign(g) wherever the oracle gradient is not tiny.
"""
import numpy as np
import pytest

import paper_1003_4570_amd as tbh
from oracle import conv as Cv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tbh.Context(0)


def _setup(grid, seed, cin=1, n_layers=4):
    rng = np.random.default_rng(seed)
    params = Cv.init_params(rng, channels=32, in_channels=cin, n_layers=n_layers)
    for W, b in params:
        b += (rng.standard_normal(b.shape) * 0.05).astype(np.float32)
    nx, ny, nz = grid
    x = np.zeros((cin, nz, ny, nx), np.float32)
    idx = rng.choice(nz * ny * nx, size=max(3, nz * ny * nx // 60), replace=False)
    x[0].ravel()[idx] = 1.0
    for c in range(1, cin):
        x[c] = rng.standard_normal((nz, ny, nx)).astype(np.float32) * 0.3
    t = rng.standard_normal((nz, ny, nx)).astype(np.float32) * 0.5
    return params, (x if cin > 1 else x[0]), t


def _halfp(params):
    return [(W.astype(np.float16).astype(np.float64), b.astype(np.float16).astype(np.float64)) for W, b in params]


@pytest.mark.parametrize("grid,cin,dil", [((12, 12, 32), 1, (1, 2, 4, 1)), ((7, 5, 9), 1, (1, 2, 4, 1)),
                                          ((32, 32, 24), 1, (1, 2, 4, 1)), ((12, 12, 32), 4, (1, 2, 4, 1)),
                                          ((7, 5, 9), 4, (1, 2, 4, 1)), ((12, 12, 32), 4, (1, 2, 4, 8, 2, 1)),
                                          ((7, 5, 9), 1, (2, 5))])
def test_forward_parity(ctx, grid, cin, dil):
    import torch
    params, x, _ = _setup(grid, 1, cin, len(dil))
    net = tbh.Net(ctx, grid, in_channels=cin, dilations=dil)
    net.set_params(tbh.flatten_params(params))
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    xr = x.astype(np.float64) if cin > 1 else x[None].astype(np.float64)
    yr, _ = Cv.forward(xr.astype(np.float16).astype(np.float64), _halfp(params), half_acts=True, dilations=dil)
    err = np.linalg.norm(y - yr[0]) / np.linalg.norm(yr[0])
    print(grid, "forward rel err", err, flush=True)
    assert err < 1e-3
    # parameters round-trip in canonical order
    assert np.array_equal(net.get_params(), tbh.flatten_params(params))


@pytest.mark.parametrize("cin,grid,dil,bar", [(1, (12, 12, 32), (1, 2, 4, 1), 1e-3), (4, (12, 12, 32), (1, 2, 4, 1), 1e-3),
                                              (4, (32, 32, 40), (1, 2, 4, 1), 6e-3)],
                         ids=["cin1", "cin4", "cin4_multichunk"])
def test_gradient_parity(ctx, cin, grid, dil, bar):
    """Gradients of four-layer nets with random weights against the oracle
    (FP16-rounded weights and activations, FP64 arithmetic).  The device
    accumulates in FP32 before it rounds each activation and upstream
    gradient to FP16, so a few roundings fall on the other side of an FP16
    boundary; the first layer's weight gradient, a sum over every voxel of
    zero-mean inputs times those gradients, collects the most of it and
    more on a larger grid.  A CPU model of exactly that arithmetic (FP32
    sums, FP16 storage) differs from the oracle there by 3.6e-4 on the
    12 x 12 x 32 grid and 2.2e-3 on the 32 x 32 x 40 grid, the bars are
    set above those.  The 32 x 32 x 40 grid (the 8 x 8 x 60-cell slab's
    cross-section) has 640 chunks of 64 voxels, more than the 256
    weight-gradient workgroups, so each workgroup accumulates several;
    exactly representable data (below) checks the same kernels to 1e-6 at
    any depth."""
    import torch
    params, x, t = _setup(grid, 2, cin, len(dil))
    net = tbh.Net(ctx, grid, in_channels=cin, dilations=dil)
    net.set_params(tbh.flatten_params(params))
    g, loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    hp = _halfp(params)
    xr = (x.astype(np.float64) if cin > 1 else x[None].astype(np.float64)).astype(np.float16).astype(np.float64)
    out, cache = Cv.forward(xr, hp, half_acts=True, dilations=dil)
    lo, dout = Cv.mse(out, t[None].astype(np.float64))
    gr = Cv.backward(hp, cache, dout)
    assert loss == pytest.approx(lo, rel=1e-3)
    G = tbh.unflatten_params(g, in_channels=cin, n_layers=len(dil))
    for li in range(len(dil)):
        for k in range(2):
            ref = gr[li][k]
            err = np.linalg.norm(G[li][k] - ref) / max(np.linalg.norm(ref), 1e-30)
            print("layer", li, "W" if k == 0 else "b", "grad rel err", err, flush=True)
            assert err < bar


def _setup_exact(grid, seed, cin, nl):
    """Sparse weights in {-1, 0, 1} (1 % non-zero), integer inputs, biases,
    targets and loss weights: every activation and upstream gradient is a
    small integer, exact in FP16 storage and FP32 accumulation, so device
    and oracle must agree to the rounding of the final sums whatever the
    depth."""
    rng = np.random.default_rng(seed)
    params = []
    for li in range(nl):
        co = 1 if li == nl - 1 else 32
        ci = cin if li == 0 else 32
        W = rng.choice([-1.0, 1.0], size=(co, ci, 3, 3, 3)) * (rng.random((co, ci, 3, 3, 3)) < 0.01)
        params.append((W, rng.integers(-1, 2, co).astype(np.float64)))
    nx, ny, nz = grid
    x = rng.integers(-2, 3, (cin, nz, ny, nx)).astype(np.float32)
    t = rng.integers(-4, 5, (nz, ny, nx)).astype(np.float32)
    w = rng.integers(1, 4, (nz, ny, nx)).astype(np.float32)
    return params, x, t, w


@pytest.mark.parametrize("cin,dil,grid", [(4, (1, 2, 4, 8, 2, 1), (12, 12, 32)), (1, (3, 1), (12, 12, 32)),
                                          (4, (1, 2, 4, 1), (12, 12, 32)), (4, (1, 2, 4, 8, 2, 1), (32, 32, 40))],
                         ids=["deep", "two_layers", "four_layers", "deep_multichunk"])
def test_gradient_exact_deep_and_weighted(ctx, cin, dil, grid):
    """Any depth and dilation list, weighted loss, on exactly representable
    values: forward and every layer's gradients equal the oracle's to 1e-6.
    The 32 x 32 x 40 grid has more 64-voxel chunks than weight-gradient
    workgroups, so each workgroup accumulates several."""
    import torch
    nl = len(dil)
    params, x, t, w = _setup_exact(grid, 7, cin, nl)
    out, cache = Cv.forward(x.astype(np.float64), params, dilations=dil)
    lo, dout = Cv.mse(out, t[None].astype(np.float64), w[None].astype(np.float64))
    gr = Cv.backward(params, cache, dout)
    # the premise: FP16 storage of activations and gradients changes nothing
    out16, cache16 = Cv.forward(x.astype(np.float64), params, half_acts=True, dilations=dil)
    gr16 = Cv.backward(params, cache16, dout * out.size, half_grads=True)
    assert np.array_equal(out16, out)
    assert all(np.abs(g16[0] / out.size - g[0]).max() <= 1e-12 * max(1.0, np.abs(g[0]).max())
               for g16, g in zip(gr16, gr))
    assert all((np.abs(g[0]) > 0).sum() > 100 for g in gr[:-1])
    net = tbh.Net(ctx, grid, in_channels=cin, dilations=dil)
    net.set_params(tbh.flatten_params(params))
    net.set_loss_weights(torch.from_numpy(w).cuda())
    xd = torch.from_numpy(x if cin > 1 else x[0]).contiguous().cuda()
    y = net.forward(xd).cpu().numpy()
    assert np.abs(y - out[0]).max() <= 1e-6 * max(1.0, np.abs(out).max())
    g, loss = net.gradients(xd, torch.from_numpy(t).cuda())
    assert loss == pytest.approx(lo, rel=1e-6)
    G = tbh.unflatten_params(g, in_channels=cin, n_layers=nl)
    for li in range(nl):
        for k in range(2):
            ref = gr[li][k]
            err = np.linalg.norm(G[li][k] - ref) / max(np.linalg.norm(ref), 1e-30)
            print("layer", li, "W" if k == 0 else "b", "grad rel err", err, flush=True)
            assert err < 1e-6
    net.set_loss_weights(None)
    _, loss1 = net.gradients(xd, torch.from_numpy(t).cuda())
    assert loss1 == pytest.approx(Cv.mse(out, t[None].astype(np.float64))[0], rel=1e-6)


def test_adam_first_step_and_loss_decreases(ctx):
    import torch
    grid = (12, 12, 32)
    params, x, t = _setup(grid, 3)
    net = tbh.Net(ctx, grid)
    w0 = tbh.flatten_params(params)
    net.set_params(w0)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    lr = 1e-3
    l0 = net.train_step([xd], [td], lr=lr)
    w1 = net.get_params()
    hp = _halfp(params)
    out, cache = Cv.forward(x[None].astype(np.float64), hp, half_acts=True)
    _, dout = Cv.mse(out, t[None].astype(np.float64))
    gref = tbh.flatten_params([(dW, db) for dW, db in Cv.backward(hp, cache, dout)]).astype(np.float64)
    big = np.abs(gref) > 1e-2 * np.abs(gref).max()
    want = w0.astype(np.float64) - lr * np.sign(gref)
    assert np.abs(w1[big] - want[big]).max() < 1e-6 + 1e-6 * np.abs(want[big]).max()
    losses = [l0]
    for _ in range(30):
        losses.append(net.train_step([xd], [td], lr=lr))
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.8 * losses[0]
