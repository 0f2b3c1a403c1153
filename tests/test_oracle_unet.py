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


def test_adam_first_step_is_signed_learning_rate():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    w = rng.normal(size=20)
    g = rng.normal(size=20)
    w1, m1, v1 = U.adam(w, g, np.zeros(20), np.zeros(20), 1e-2, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(w - w1, 1e-2 * np.sign(g), atol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 1e-3 * g * g)
    # a constant gradient keeps the corrected step at lr * sign(g) for every step
    w2, m2, v2 = U.adam(w1, g, m1, v1, 1e-2, 0.9, 0.999, 1e-12, 2)
    assert np.allclose(w1 - w2, 1e-2 * np.sign(g), atol=1e-10)


def test_block_mean_against_loops_and_invariants():
    rng = np.random.default_rng(4)
    f = rng.normal(size=(4, 6, 8))
    mask = rng.uniform(size=f.shape) > 0.3
    out = U.block_mean([f, 2 * f], mask, 2)
    z, y, x = 1, 2, 3
    vals = [f[2 * z + a, 2 * y + b, 2 * x + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)
            if mask[2 * z + a, 2 * y + b, 2 * x + c]]
    assert out[z, y, x, 0] == pytest.approx(np.mean(vals))
    assert out[z, y, x, 1] == pytest.approx(2 * np.mean(vals))
    assert out[z, y, x, 2] == pytest.approx(len(vals) / 8)
    # full mask: the data-weighted mean over all blocks is the global mean
    full = U.block_mean([f], None, 2)
    assert full[..., 0].mean() == pytest.approx(f.mean())
    assert np.all(full[..., 1] == 1.0)


def test_upsample_is_exact_on_linear_fields_up_to_the_edge():
    cz, cy, cx = np.meshgrid(np.arange(3.0), np.arange(4.0), np.arange(5.0), indexing="ij")
    coarse = 0.5 + 2.0 * cx - 1.5 * cy + 0.25 * cz
    f = 4
    up = U.upsample_linear(coarse, f)
    assert up.shape == (12, 16, 20)
    # every fine centre, the half coarse cell beyond the outermost coarse
    # centres included: the linear field at its coarse coordinate
    k, j, i = np.meshgrid(np.arange(12.0), np.arange(16.0), np.arange(20.0), indexing="ij")
    u = [(v + 0.5) / f - 0.5 for v in (k, j, i)]
    assert np.abs(up - (0.5 + 2.0 * u[2] - 1.5 * u[1] + 0.25 * u[0])).max() < 1e-12
    assert up[0, 0, 0] == pytest.approx(0.5 - 2.0 * 0.375 + 1.5 * 0.375 - 0.25 * 0.375)
    assert np.allclose(U.upsample_linear(np.full((2, 3), 7.0), 3), 7.0)
    # an axis of one coarse cell is constant along it
    assert np.allclose(U.upsample_linear(np.arange(3.0)[None, :], 2)[:, 0], -0.25)


def test_upsample_against_a_direct_double_loop():
    """Interpolation weights written out per fine cell (2-D), independently
    of the per-axis form."""
    rng = np.random.default_rng(5)
    c = rng.normal(size=(3, 4))
    f = 2
    up = U.upsample_linear(c, f)
    for y in range(6):
        for x in range(8):
            uy, ux = (y + 0.5) / f - 0.5, (x + 0.5) / f - 0.5
            y0, x0 = min(max(int(np.floor(uy)), 0), 1), min(max(int(np.floor(ux)), 0), 2)
            ty, tx = uy - y0, ux - x0
            ref = ((1 - ty) * (1 - tx) * c[y0, x0] + (1 - ty) * tx * c[y0, x0 + 1] + ty * (1 - tx) * c[y0 + 1, x0] +
                   ty * tx * c[y0 + 1, x0 + 1])
            assert up[y, x] == pytest.approx(ref, abs=1e-12)
