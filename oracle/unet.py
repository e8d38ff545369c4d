"""Float64 NumPy reference of the warm-start network (forward and backward).

TEST INFRASTRUCTURE: part of the CPU oracle (see oracle/__init__.py).  It
checks the GPU network kernels; its own backward pass is pinned by finite
differences in the tests.

The network maps three input fields on an H x W grid -- log-permeability
lnK, saturation S and the proximity of the nearest Dirichlet wall,
exp(-d / 16) with d = min(x + 1/2, W - x - 1/2) in nodes -- to a pressure
estimate used as the starting pressure of the lattice Boltzmann iteration
(the iteration itself is unchanged and runs to the same tolerance).  Inputs
and output are stated per node, so a network trained on one grid size applies
to others: the deviation of P from the linear profile scales like the mean
gradient 1/W.
It is a convolutional encoder-decoder with `levels` resolution levels and
`base` channels at the top level (base * 2^l at level l):

  encoder level l:  conv3x3 -> ReLU -> conv3x3 -> ReLU   (skip s_l)
                    2x2 average pooling between levels
  decoder level l:  nearest 2x upsampling of the level below,
                    channel concatenation [upsampled, s_l],
                    conv3x3 -> ReLU -> conv3x3 -> ReLU
  head:             conv3x3 (base -> 1), no activation
  output:           P = (1 - (x + 1/2)/W) + (scale / W) * head

All 3x3 convolutions use zero padding ("same" size) and a bias.  Tensors are
laid out [N][H][W][C].  Parameters are one flat float vector: for every
convolution in the order of `layers()`, its weights [Co][3][3][Ci] followed
by its bias [Co].
"""
import numpy as np


def layers(base=32, levels=4, cin=3):
    """(ci, co, relu) of every convolution, in forward order."""
    out = []
    c = [base * 2 ** l for l in range(levels)]
    prev = cin
    for l in range(levels):
        out.append((prev, c[l], True))
        out.append((c[l], c[l], True))
        prev = c[l]
    for l in range(levels - 2, -1, -1):
        out.append((c[l + 1] + c[l], c[l], True))
        out.append((c[l], c[l], True))
    out.append((c[0], 1, False))
    return out


def n_params(base=32, levels=4):
    return sum(co * 9 * ci + co for ci, co, _ in layers(base, levels))


def init_params(base=32, levels=4, seed=0):
    """He-normal weights, zero biases (float32-representable values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, relu in layers(base, levels):
        std = np.sqrt(2.0 / (9 * ci)) if relu else np.sqrt(1.0 / (9 * ci))
        parts.append((rng.standard_normal((co, 3, 3, ci)) * std).ravel())
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def unpack(theta, base=32, levels=4):
    ws, off = [], 0
    for ci, co, _ in layers(base, levels):
        w = theta[off:off + co * 9 * ci].reshape(co, 3, 3, ci)
        off += co * 9 * ci
        b = theta[off:off + co]
        off += co
        ws.append((w, b))
    return ws


def _patches(x):
    """[N,H,W,C] -> [N,H,W,3,3,C] zero-padded 3x3 neighbourhoods."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    out = np.empty((N, H, W, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            out[:, :, :, ky, kx] = xp[:, ky:ky + H, kx:kx + W]
    return out


def conv(x, w, b):
    """y[n,i,j,o] = b[o] + sum_{ky,kx,c} w[o,ky,kx,c] x[n, i+ky-1, j+kx-1, c]."""
    return np.einsum("nhwykc,oykc->nhwo", _patches(x), w, optimize=True) + b


def conv_backward(x, w, dy):
    """Gradients of conv() with respect to x, w and b."""
    N, H, W, C = x.shape
    dw = np.einsum("nhwykc,nhwo->oykc", _patches(x), dy, optimize=True)
    db = dy.sum(axis=(0, 1, 2))
    # dx[n, i', j', c] = sum_{ky,kx,o} dy[n, i'-ky+1, j'-kx+1, o] w[o,ky,kx,c]
    dyp = np.zeros((N, H + 2, W + 2, dy.shape[-1]))
    dyp[:, 1:-1, 1:-1] = dy
    dx = np.zeros_like(x)
    for ky in range(3):
        for kx in range(3):
            dx += np.einsum("nhwo,oc->nhwc", dyp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W], w[:, ky, kx, :])
    return dx, dw, db


def pool(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def inputs(lnK, S):
    """[N,H,W] fields -> [N,H,W,3] network input (lnK, S, wall proximity)."""
    N, H, W = lnK.shape
    x = np.arange(W) + 0.5
    d = np.minimum(x, W - x)
    wall = np.broadcast_to(np.exp(-d / 16.0), (N, H, W))
    return np.stack([lnK, S, wall], axis=-1)


def forward(theta, lnK, S, scale, base=32, levels=4, keep=False):
    """Predicted pressure [N,H,W]; with keep=True also the tape for backward()."""
    ws = unpack(theta, base, levels)
    x = inputs(lnK, S)
    tape = []
    li = 0

    def cr(x, relu):
        nonlocal li
        w, b = ws[li]
        li += 1
        z = conv(x, w, b)
        y = np.maximum(z, 0.0) if relu else z
        tape.append((x, z, relu))
        return y

    skips = []
    h = x
    for l in range(levels):
        if l > 0:
            h = pool(h)
        h = cr(h, True)
        h = cr(h, True)
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        h = np.concatenate([up(h), skips[l]], axis=-1)
        h = cr(h, True)
        h = cr(h, True)
    h = cr(h, False)
    N, H, W = lnK.shape
    ramp = 1.0 - (np.arange(W) + 0.5) / W
    P = ramp + (scale / W) * h[..., 0]
    return (P, tape) if keep else P


def coarsen(x, f):
    """Block mean of [N, H, W] over f x f blocks."""
    N, H, W = x.shape
    return x.reshape(N, H // f, f, W // f, f).mean(axis=(2, 4))


def interpolate(d, f):
    """Bilinear interpolation of node-centred values d [N, h, w] to the grid
    refined by f: fine node x sits at coarse coordinate (x + 1/2)/f - 1/2;
    coordinates outside [0, w - 1] take the edge value."""
    def axis(n):
        u = (np.arange(n * f) + 0.5) / f - 0.5
        u = np.clip(u, 0.0, n - 1)
        i0 = np.minimum(np.floor(u).astype(int), n - 1)
        i1 = np.minimum(i0 + 1, n - 1)
        return i0, i1, u - i0
    N, h, w = d.shape
    y0, y1, ty = axis(h)
    x0, x1, tx = axis(w)
    rows = d[:, y0, :] * (1 - ty)[None, :, None] + d[:, y1, :] * ty[None, :, None]
    return rows[:, :, x0] * (1 - tx) + rows[:, :, x1] * tx


def predict(theta, lnK, S, scale, factor=1, base=32, levels=4):
    """Initial pressure of an H x W grid; for factor > 1 the network sees the
    fields coarsened by `factor` and its deviation from the coarse linear
    profile is interpolated to the fine grid and added to the fine profile."""
    if factor == 1:
        return forward(theta, lnK, S, scale, base, levels)
    W = lnK.shape[2]
    Pc = forward(theta, coarsen(lnK, factor), coarsen(S, factor), scale, base, levels)
    wc = W // factor
    dev = Pc - (1.0 - (np.arange(wc) + 0.5) / wc)
    return (1.0 - (np.arange(W) + 0.5) / W) + interpolate(dev, factor)


def loss_and_grad(theta, lnK, S, P_target, scale, base=32, levels=4, weight=None):
    """Weighted mean squared error of the predicted pressure,
    L = (1 / (N H W)) sum_n weight[n] sum_nodes (P - P_target)^2 (weight None:
    all ones), and its gradient (flat)."""
    ws = unpack(theta, base, levels)
    P, tape = forward(theta, lnK, S, scale, base, levels, keep=True)
    r = P - P_target
    wn = np.ones(r.shape[0]) if weight is None else np.asarray(weight, float)
    loss = float(np.sum(wn[:, None, None] * r * r) / r.size)
    dP = 2.0 * wn[:, None, None] * r / r.size
    grads = [None] * len(ws)
    li = len(ws) - 1

    def cb(dy):
        nonlocal li
        x, z, relu = tape[li]
        if relu:
            dy = dy * (z > 0)
        dx, dw, db = conv_backward(x, ws[li][0], dy)
        grads[li] = (dw, db)
        li -= 1
        return dx

    dh = np.zeros(tape[-1][1].shape)
    dh[..., 0] = (scale / lnK.shape[2]) * dP
    dh = cb(dh)
    c = [base * 2 ** l for l in range(levels)]
    dskips = [None] * levels
    for l in range(0, levels - 1):
        dh = cb(dh)
        dh = cb(dh)
        cu = c[l + 1]
        dskips[l] = dh[..., cu:]
        dh = up_backward(dh[..., :cu])
    for l in range(levels - 1, -1, -1):
        if dskips[l] is not None and l < levels - 1:
            dh = dh + dskips[l]
        dh = cb(dh)
        dh = cb(dh)
        if l > 0:
            dh = pool_backward(dh)
    flat = np.concatenate([np.concatenate([dw.ravel(), db]) for dw, db in grads])
    return loss, flat
