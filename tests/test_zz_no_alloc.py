"""lbtp_nn_predict_noalloc (the warm-start network's inference with its
buffers in a static device array) against lbtp_nn_predict, through the C ABI:
two calls in a row, the second on a smaller input, must give the same
pressure bit for bit (same kernels in the same order); a shape too large for
the array is rejected before anything runs."""
import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu

BASE, LEVELS, SCALE = 32, 4, 3.2


def _inputs(N, H, W, seed):
    import torch
    rng = np.random.default_rng(seed)
    lnK = torch.from_numpy(rng.standard_normal((N, H, W)).astype(np.float32)).cuda()
    S = torch.from_numpy(rng.uniform(0, 1, (N, H, W)).astype(np.float32)).cuda()
    return lnK, S


def test_noalloc_predict_equals_predict():
    import torch
    from paper_1808_07554_amd import lbtp
    th = unet.init_params(BASE, LEVELS, seed=5)
    th = th + 0.01 * np.random.default_rng(6).standard_normal(th.size)
    net = lbtp.WarmStartNet(BASE, LEVELS, SCALE)
    net.set_params(th.astype(np.float32))
    # the first call is the larger one, so the second finds the array holding
    # the first call's values beyond its own buffers
    for (N, H, W, factor, seed) in [(2, 512, 256, 4, 1), (1, 64, 128, 2, 2), (1, 32, 32, 1, 3)]:
        lnK, S = _inputs(N, H, W, seed)
        ref = net.predict(lnK, S, factor)
        P = torch.full_like(lnK, float("nan"))
        net.predict_noalloc(lnK, S, P, factor)
        torch.cuda.synchronize()
        assert torch.isfinite(P).all()
        assert torch.equal(P, ref), (N, H, W, factor, float((P - ref).abs().max()))
    # too large for the static array: rejected, output untouched
    lnK, S = _inputs(1, 512, 512, 4)
    P = torch.zeros_like(lnK)
    with pytest.raises(lbtp.LbtpError):
        net.predict_noalloc(lnK, S, P, 1)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(P)) == 0
    net.close()
