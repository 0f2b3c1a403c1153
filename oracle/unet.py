"""FP64 reference of the warm-start network's layers, forward and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain direct
definitions in NumPy, channels-last arrays [N, D, H, W, C]:

* conv3: 3x3x3 convolution, stride 1, zero padding 1, weights [27, Cin, Cout]
  with tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), plus bias; optional ReLU.
* upconv: 2x2x2 transposed convolution with stride 2, weights [8, Cin, Cout]
  with tap q = 4 qz + 2 qy + qx: out[2p + q] = sum_ci in[p, ci] W[q, ci, :].
* pool: 2x2x2 average pooling.
* head: 1x1x1 convolution to one channel, FP output.
* mse: mean of (pred - target)^2 over the cells where the mask is set.

Backward passes are the derivatives of these definitions written out (dx,
dW, db); they are pinned against central finite differences in
tests/test_oracle_unet.py.
"""

from __future__ import annotations

import numpy as np

TAPS3 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """y[n, z, y, x] = x[n, z + dz, y + dy, x + dx], zero outside."""
    n, D, H, W, C = x.shape
    out = np.zeros_like(x)
    zs, ys, xs = slice(max(0, -dz), D - max(0, dz)), slice(max(0, -dy), H - max(0, dy)), slice(max(0, -dx), W - max(0, dx))
    zt, yt, xt = slice(max(0, dz), D + min(0, dz)), slice(max(0, dy), H + min(0, dy)), slice(max(0, dx), W + min(0, dx))
    out[:, zs, ys, xs] = x[:, zt, yt, xt]
    return out


def conv3(x, W, b, relu=False):
    y = np.zeros(x.shape[:4] + (W.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS3):
        y += _shift(x, dz, dy, dx) @ W[t]
    y += b
    return np.maximum(y, 0.0) if relu else y


def conv3_backward(x, W, gy):
    """Gradients of y = conv3(x, W, b) (before any activation) given dL/dy."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(TAPS3):
        xs = _shift(x, dz, dy, dx)
        gW[t] = xs.reshape(-1, x.shape[-1]).T @ gy.reshape(-1, gy.shape[-1])
        gx += _shift(gy @ W[t].T, -dz, -dy, -dx)
    gb = gy.reshape(-1, gy.shape[-1]).sum(axis=0)
    return gx, gW, gb


def upconv(x, W, b):
    n, D, H, Wd, _ = x.shape
    y = np.zeros((n, 2 * D, 2 * H, 2 * Wd, W.shape[2]))
    for q in range(8):
        qz, qy, qx = q >> 2, (q >> 1) & 1, q & 1
        y[:, qz::2, qy::2, qx::2] = x @ W[q]
    return y + b


def upconv_backward(x, W, gy):
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for q in range(8):
        qz, qy, qx = q >> 2, (q >> 1) & 1, q & 1
        g = gy[:, qz::2, qy::2, qx::2]
        gx += g @ W[q].T
        gW[q] = x.reshape(-1, x.shape[-1]).T @ g.reshape(-1, g.shape[-1])
    gb = gy.reshape(-1, gy.shape[-1]).sum(axis=0)
    return gx, gW, gb


def pool(x):
    n, D, H, W, C = x.shape
    return x.reshape(n, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool_backward(gy):
    g = np.repeat(np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2), 2, axis=3)
    return g / 8.0


def head(x, w, b):
    return x @ w + b


def head_backward(x, w, gy):
    return np.outer(gy.reshape(-1), w).reshape(x.shape), x.reshape(-1, x.shape[-1]).T @ gy.reshape(-1), gy.sum()


def mse(pred, target, mask):
    m = mask.astype(np.float64)
    cnt = m.sum()
    d = (pred - target) * m
    return float((d * d).sum() / cnt), 2.0 * d / cnt


def adam(w, g, m, v, lr, beta1, beta2, eps, step):
    """One Adam step (Kingma and Ba, Algorithm 1) with bias-corrected moments;
    returns the new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def block_mean(fields, mask, factor):
    """Network input from solver-grid fields (storage order [z, y, x] or
    [y, x]): per factor-sized block, the mean of each field over the block's
    data cells (0 if none) and the fraction of data cells."""
    nd = fields[0].ndim
    m = np.ones(fields[0].shape, bool) if mask is None else np.asarray(mask, bool)
    cshape = tuple(s // factor for s in fields[0].shape)
    out = np.zeros(cshape + (len(fields) + 1,))
    for idx in np.ndindex(*cshape):
        sl = tuple(slice(i * factor, (i + 1) * factor) for i in idx)
        mb = m[sl]
        cnt = mb.sum()
        for k, f in enumerate(fields):
            out[idx + (k,)] = f[sl][mb].sum() / cnt if cnt else 0.0
        out[idx + (len(fields),)] = cnt / factor ** nd
    return out


def upsample_linear(coarse, factor):
    """Cell-centred multilinear interpolation of a coarse field onto a grid
    `factor` times finer along every axis, one 1-D interpolation per axis:
    a fine centre at coarse coordinate u = (i + 1/2) / factor - 1/2 takes the
    straight line through the two coarse centres around it, and the line
    through the two outermost ones beyond them (so a field linear in the
    coordinates is reproduced up to the grid's edge); an axis of one coarse
    cell is constant."""
    out = np.asarray(coarse, float)
    for ax in range(out.ndim):
        n = out.shape[ax]
        u = (np.arange(n * factor) + 0.5) / factor - 0.5
        if n == 1:
            out = np.repeat(out, factor, axis=ax)
            continue
        i0 = np.clip(np.floor(u).astype(int), 0, n - 2)
        t = u - i0
        a = np.take(out, i0, axis=ax)
        b = np.take(out, i0 + 1, axis=ax)
        shape = [1] * out.ndim
        shape[ax] = -1
        t = t.reshape(shape)
        out = a + t * (b - a)
    return out
