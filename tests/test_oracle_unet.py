"""Pins of the float64 reference network (oracle/unet.py): the convolution
against scipy's correlate, pooling/upsampling identities, and the
hand-written backward pass against central finite differences."""
import numpy as np
import scipy.ndimage as ndi

from oracle import unet

RNG = np.random.default_rng(7)


def test_conv_matches_scipy_correlate():
    x = RNG.standard_normal((2, 7, 9, 3))
    w = RNG.standard_normal((4, 3, 3, 3))
    b = RNG.standard_normal(4)
    y = unet.conv(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(ndi.correlate(x[n, :, :, c], w[o, :, :, c], mode="constant", cval=0.0) for c in range(3))
            assert np.allclose(y[n, :, :, o], ref + b[o], atol=1e-12)


def test_pool_up_adjoint():
    x = RNG.standard_normal((2, 8, 6, 3))
    y = RNG.standard_normal((2, 4, 3, 3))
    # <pool x, y> = <x, pool^T y> and <up y, x> = <y, up^T x>
    assert np.isclose(np.sum(unet.pool(x) * y), np.sum(x * unet.pool_backward(y)))
    assert np.isclose(np.sum(unet.up(y) * x), np.sum(y * unet.up_backward(x)))
    assert np.allclose(unet.pool(unet.up(y)), y)


def test_coarsen_and_interpolate():
    # block mean: constants stay, nearest-upsampled fields come back exactly
    y = RNG.standard_normal((2, 5, 3))
    up = np.repeat(np.repeat(y, 4, axis=1), 4, axis=2)
    assert np.allclose(unet.coarsen(up, 4), y)
    assert np.allclose(unet.coarsen(np.full((1, 8, 12), 2.5), 4), 2.5)
    # bilinear refinement with node-centre alignment and edge clamping is
    # scipy's order-1 zoom in grid mode with 'nearest' edges
    d = RNG.standard_normal((2, 6, 5))
    for f in (2, 4, 16):
        got = unet.interpolate(d, f)
        ref = np.stack([ndi.zoom(d[n], f, order=1, mode="nearest", grid_mode=True) for n in range(2)])
        assert got.shape == (2, 6 * f, 5 * f) and np.allclose(got, ref, atol=1e-12)
    # linear functions are reproduced exactly away from the clamped edges
    h, w, f = 6, 5, 4
    Y, X = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    lin = (0.3 + 0.7 * X - 0.2 * Y)[None].astype(float)
    fine = unet.interpolate(lin, f)
    v = (np.arange(h * f) + 0.5) / f - 0.5
    u = (np.arange(w * f) + 0.5) / f - 0.5
    inner = (slice(None), slice(f // 2, h * f - f // 2), slice(f // 2, w * f - f // 2))
    ref = 0.3 + 0.7 * u[None, None, :] - 0.2 * v[None, :, None]
    assert np.allclose(fine[inner], np.broadcast_to(ref, fine.shape)[inner], atol=1e-12)


def test_coarse_predict_keeps_the_linear_profile():
    # with a zero network the prediction is the fine linear profile for any factor
    th = np.zeros(unet.n_params(4, 2))
    lnK = RNG.standard_normal((1, 16, 32))
    for f in (1, 2, 4):
        P = unet.predict(th, lnK, lnK, 1.0, f, base=4, levels=2)
        assert np.allclose(P, 1.0 - (np.arange(32) + 0.5) / 32)


def test_layer_list_and_parameter_count():
    L = unet.layers(32, 4)
    assert len(L) == 15
    assert L[0] == (3, 32, True) and L[7] == (256, 256, True) and L[8] == (384, 128, True) and L[-1] == (32, 1, False)
    assert unet.n_params(32, 4) == sum(co * 9 * ci + co for ci, co, _ in L)


def test_backward_matches_finite_differences():
    base, levels = 4, 3
    N, H, W = 2, 8, 8
    theta = unet.init_params(base, levels, seed=3)
    theta = theta + 0.05 * RNG.standard_normal(theta.size)      # non-zero biases too
    lnK = RNG.standard_normal((N, H, W))
    S = RNG.uniform(0, 1, (N, H, W))
    Pt = RNG.standard_normal((N, H, W)) * 0.1 + 0.5
    scale = 0.3
    wts = np.array([0.5, 2.0])
    loss, g = unet.loss_and_grad(theta, lnK, S, Pt, scale, base, levels, weight=wts)

    def wmse(th):
        r = unet.forward(th, lnK, S, scale, base, levels) - Pt
        return np.mean(wts[:, None, None] * r * r)
    assert np.isclose(loss, wmse(theta))
    idx = RNG.choice(theta.size, 60, replace=False)
    eps = 1e-6
    bad = 0
    for i in idx:
        tp = theta.copy()
        tp[i] += eps
        tm = theta.copy()
        tm[i] -= eps
        fp = wmse(tp)
        fm = wmse(tm)
        fd = (fp - fm) / (2 * eps)
        if abs(fd - g[i]) > 1e-6 * max(1.0, abs(fd)) + 1e-9:
            bad += 1
    # a parameter whose perturbation moves a ReLU input across zero may disagree
    assert bad <= 1, bad
