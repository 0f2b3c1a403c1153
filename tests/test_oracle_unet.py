"""Pins of the FP64 layer oracle of the warm-start network: every backward
pass against central finite differences of its forward pass, and the
forward passes against direct per-element loops."""

import numpy as np
import pytest

from oracle import unet as U


def _fd(f, x, eps=1e-6, idx=None):
    """Central finite difference of scalar f at a few entries of x."""
    g = {}
    for i in idx:
        x0 = x[i]
        x[i] = x0 + eps
        fp = f()
        x[i] = x0 - eps
        fm = f()
        x[i] = x0
        g[i] = (fp - fm) / (2 * eps)
    return g


def _pick(shape, k, rng):
    return [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(k)]


def test_conv3_forward_is_direct_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(1, 4, 3, 5, 2))
    W = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    y = U.conv3(x, W, b)
    for (z, yy, xx) in [(0, 0, 0), (3, 2, 4), (1, 1, 2)]:
        for co in range(3):
            acc = b[co]
            for t, (dz, dy, dx) in enumerate(U.TAPS3):
                zz, y2, x2 = z + dz, yy + dy, xx + dx
                if 0 <= zz < 4 and 0 <= y2 < 3 and 0 <= x2 < 5:
                    acc += x[0, zz, y2, x2] @ W[t][:, co]
            assert y[0, z, yy, xx, co] == pytest.approx(acc, abs=1e-12)


def test_conv3_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 4, 5, 3))
    W = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=2)
    R = rng.normal(size=(2, 3, 4, 5, 2))
    loss = lambda: float((U.conv3(x, W, b) * R).sum())  # noqa: E731
    gx, gW, gb = U.conv3_backward(x, W, R)
    for i, v in _fd(loss, x, idx=_pick(x.shape, 6, rng)).items():
        assert gx[i] == pytest.approx(v, rel=1e-6, abs=1e-8)
    for i, v in _fd(loss, W, idx=_pick(W.shape, 6, rng)).items():
        assert gW[i] == pytest.approx(v, rel=1e-6, abs=1e-8)
    for i, v in _fd(loss, b, idx=[(0,), (1,)]).items():
        assert gb[i] == pytest.approx(v, rel=1e-6)


def test_upconv_pool_head_backward_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 2, 3, 2, 3))
    W = rng.normal(size=(8, 3, 2))
    b = rng.normal(size=2)
    R = rng.normal(size=(1, 4, 6, 4, 2))
    loss = lambda: float((U.upconv(x, W, b) * R).sum())  # noqa: E731
    gx, gW, gb = U.upconv_backward(x, W, R)
    for i, v in _fd(loss, x, idx=_pick(x.shape, 5, rng)).items():
        assert gx[i] == pytest.approx(v, rel=1e-6, abs=1e-8)
    for i, v in _fd(loss, W, idx=_pick(W.shape, 5, rng)).items():
        assert gW[i] == pytest.approx(v, rel=1e-6, abs=1e-8)
    # pool
    xp = rng.normal(size=(1, 4, 2, 6, 3))
    Rp = rng.normal(size=(1, 2, 1, 3, 3))
    lp = lambda: float((U.pool(xp) * Rp).sum())  # noqa: E731
    gp = U.pool_backward(Rp)
    for i, v in _fd(lp, xp, idx=_pick(xp.shape, 5, rng)).items():
        assert gp[i] == pytest.approx(v, rel=1e-6, abs=1e-9)
    # head and the masked mean squared error
    xh = rng.normal(size=(1, 3, 2, 2, 4))
    w = rng.normal(size=4)
    target = rng.normal(size=(1, 3, 2, 2))
    mask = rng.uniform(size=target.shape) > 0.3
    lh = lambda: U.mse(U.head(xh, w, 0.3), target, mask)[0]  # noqa: E731
    l0, gpred = U.mse(U.head(xh, w, 0.3), target, mask)
    gxh, gw, gbh = U.head_backward(xh, w, gpred)
    for i, v in _fd(lh, xh, idx=_pick(xh.shape, 5, rng)).items():
        assert gxh[i] == pytest.approx(v, rel=1e-6, abs=1e-9)
    for i, v in _fd(lh, w, idx=[(0,), (3,)]).items():
        assert gw[i] == pytest.approx(v, rel=1e-6, abs=1e-9)
