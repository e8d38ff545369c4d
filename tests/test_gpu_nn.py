"""The warm-start network on the GPU (bf16 MFMA kernels) against the float64
reference network (oracle/unet.py, itself pinned by finite differences)."""
import numpy as np
import pytest

from oracle import unet
from tests.lbhelp import rel_l2

pytestmark = pytest.mark.gpu

BASE, LEVELS, SCALE = 32, 4, 3.2


def _data(N, H, W, seed):
    rng = np.random.default_rng(seed)
    lnK = rng.standard_normal((N, H, W)).astype(np.float32)
    S = rng.uniform(0, 1, (N, H, W)).astype(np.float32)
    x = (np.arange(W) + 0.5) / W
    P = (1 - x + 0.02 * rng.standard_normal((N, H, W))).astype(np.float32)
    return lnK, S, P


def _net(theta):
    from paper_1808_07554_amd import lbtp
    net = lbtp.WarmStartNet(BASE, LEVELS, SCALE)
    net.set_params(theta.astype(np.float32))
    return net


def _theta(seed=1):
    th = unet.init_params(BASE, LEVELS, seed=seed)
    rng = np.random.default_rng(seed + 100)
    th = th + 0.01 * rng.standard_normal(th.size)     # non-zero biases
    return th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(2, 32, 32), (1, 16, 48)])
def test_forward_matches_reference(shape):
    N, H, W = shape
    lnK, S, _ = _data(N, H, W, 3)
    th = _theta()
    net = _net(th)
    got = net.predict(lnK, S).cpu().numpy().astype(np.float64)
    ref = unet.forward(th, lnK.astype(np.float64), S.astype(np.float64), SCALE, BASE, LEVELS)
    ramp = 1.0 - (np.arange(W) + 0.5) / W
    # bf16 activations (8-bit significand) through 15 convolutions
    err = rel_l2(ref - ramp, got - ramp)
    print("forward rel err", err)
    assert err < 3e-2


@pytest.mark.parametrize("shape,factor", [((2, 64, 64), 2), ((1, 128, 64), 4), ((1, 256, 256), 16),
                                          ((2, 1024, 1024), 16)])
def test_coarse_grid_predict_matches_reference(shape, factor):
    N, H, W = shape
    lnK, S, _ = _data(N, H, W, 11)
    th = _theta(3)
    net = _net(th)
    got = net.predict(lnK, S, factor).cpu().numpy().astype(np.float64)
    ref = unet.predict(th, lnK.astype(np.float64), S.astype(np.float64), SCALE, factor, BASE, LEVELS)
    ramp = 1.0 - (np.arange(W) + 0.5) / W
    err = rel_l2(ref - ramp, got - ramp)
    print("coarse predict rel err", factor, err)
    assert err < 3e-2


@pytest.mark.parametrize("weighted", [False, True])
def test_gradients_match_reference(weighted):
    N, H, W = 2, 32, 32
    lnK, S, P = _data(N, H, W, 5)
    th = _theta(2)
    net = _net(th)
    wts = np.array([0.25, 3.0], np.float32) if weighted else None
    loss_g, g = net.loss_grad(lnK, S, P, wts)
    g = g.cpu().numpy().astype(np.float64)
    loss_r, gr = unet.loss_and_grad(th, lnK.astype(np.float64), S.astype(np.float64), P.astype(np.float64), SCALE,
                                    BASE, LEVELS, weight=wts)
    assert abs(loss_g - loss_r) <= 2e-2 * loss_r
    off = 0
    worst = 0.0
    for i, (ci, co, _) in enumerate(unet.layers(BASE, LEVELS)):
        n = co * 9 * ci + co
        a, b = gr[off:off + n], g[off:off + n]
        off += n
        e = rel_l2(a, b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        print(f"layer {i} ({ci}->{co}) rel {e:.3e} cos {cos:.5f}")
        worst = max(worst, e)
        assert cos > 0.995 and e < 0.1, (i, e, cos)
    assert rel_l2(gr, g) < 5e-2


def test_gradients_are_deterministic_and_training_reduces_loss():
    from paper_1808_07554_amd import lbtp
    N, H, W = 4, 32, 32
    lnK, S, _ = _data(N, H, W, 9)
    x = (np.arange(W) + 0.5) / W
    P = (1 - x + 0.02 * np.tanh(lnK)).astype(np.float32)     # learnable target
    net = _net(_theta(4))
    l1, g1 = net.loss_grad(lnK, S, P)
    l2, g2 = net.loss_grad(lnK, S, P)
    assert l1 == l2 and bool((g1 == g2).all())
    losses = [net.train_step(lnK, S, P, 1e-3) for _ in range(30)]
    assert losses[-1] < 0.5 * losses[0], losses[::5]


def test_bad_shapes_rejected():
    from paper_1808_07554_amd import lbtp
    net = _net(_theta())
    with pytest.raises(lbtp.LbtpError):
        net.predict(np.zeros((1, 12, 16), np.float32), np.zeros((1, 12, 16), np.float32))   # 12 % 8 != 0
    with pytest.raises(lbtp.LbtpError):
        net.predict(np.zeros((1, 64, 64), np.float32), np.zeros((1, 64, 64), np.float32), 3)   # 64 % 3 != 0
    with pytest.raises(lbtp.LbtpError):
        net.predict(np.zeros((1, 64, 64), np.float32), np.zeros((1, 64, 64), np.float32), 16)  # coarse 4 % 8 != 0
