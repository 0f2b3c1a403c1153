"""Warm-start network kernels (through the C interface) against the FP64
layer oracle.

Inputs are drawn, rounded to BF16 on the host, and handed to both sides, so
the oracle sees exactly the kernels' operands.  Bars: FP32 outputs within
2e-5 of the largest reference magnitude (FP32 accumulation over at most a
few thousand products); BF16 outputs additionally within one BF16 rounding
(2^-8 relative).  The whole-network gradient check composes the oracle's
layers in FP64, rounding to BF16 wherever the device stores an activation
or its gradient in BF16, and compares each parameter gradient in relative L2
norm (bar 1e-2: FP32 against FP64 accumulation, and the rare value that
lands on the other side of a BF16 rounding or ReLU boundary).
"""

import math

import numpy as np
import pytest
import torch

from gpu_common import DEV, announce, requires_gpu
from oracle import unet as O

pytestmark = [pytest.mark.gpu, requires_gpu]

TAPS3 = O.TAPS3
NEG3 = [(-a, -b, -c) for (a, b, c) in TAPS3]
UP8 = [(q >> 2, (q >> 1) & 1, q & 1) for q in range(8)]


def _bf(a):
    """BF16-representable float64 copy of a."""
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).double().numpy()


def _dev_bf(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).to(DEV)


def _dev_f(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def _host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def _check(got, ref, bf16_out, what):
    scale = np.abs(ref).max()
    bound = 2e-5 * scale + (2.0 ** -8) * np.abs(ref) if bf16_out else 2e-5 * scale
    err = np.abs(got - ref)
    assert np.all(err <= bound + 1e-30), f"{what}: max err {err.max():.3e} (scale {scale:.3e})"


def _wide(a, off, extra):
    """Embed channels of a [n,d,h,w,c] array at `off` in a wider buffer."""
    n, d, h, w, c = a.shape
    out = np.zeros((n, d, h, w, c + extra), np.float64)
    out[..., off:off + c] = a
    return out


@pytest.mark.parametrize("cin,cout,xoff,yoff", [(12, 24, 0, 0), (40, 72, 8, 8), (16, 8, 3, 5)])
def test_conv3_forward(cin, cout, xoff, yoff):
    from paper_2311_16935_amd import unet as U

    announce("conv3 fwd", cin, cout, xoff, yoff)
    rng = np.random.default_rng(cin + cout)
    shape = (2, 5, 6, 7)
    x = _bf(rng.normal(size=shape + (cin,)))
    W = _bf(rng.normal(size=(27, cin, cout)) / math.sqrt(27 * cin))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    xd = _dev_bf(_wide(x, xoff, 16))
    wd, bd = _dev_bf(W.transpose(0, 2, 1)), _dev_f(b)  # [tap][cout][cin]
    for relu in (False, True):
        ref = O.conv3(x, W, b, relu=relu)
        y = torch.zeros(shape + (cout + 16,), dtype=torch.bfloat16, device=DEV)
        U.pu_conv(U.tensor(xd, xoff, cin), wd, 27, TAPS3, bd, U.tensor(y, yoff, cout), shape[1:], relu=relu)
        yh = _host(y)
        _check(yh[..., yoff:yoff + cout], ref, True, f"conv relu={relu}")
        assert np.all(yh[..., :yoff] == 0) and np.all(yh[..., yoff + cout:] == 0)
    # FP32 output and accumulation into it
    y32 = torch.zeros(shape + (cout,), dtype=torch.float32, device=DEV)
    U.pu_conv(U.tensor(xd, xoff, cin), wd, 27, TAPS3, bd, U.tensor(y32), shape[1:], y_fp32=True)
    _check(_host(y32), O.conv3(x, W, b), False, "conv fp32")
    U.pu_conv(U.tensor(xd, xoff, cin), wd, 27, TAPS3, None, U.tensor(y32), shape[1:], y_fp32=True,
              accumulate=True)
    _check(_host(y32), 2 * O.conv3(x, W, b) - b, False, "conv accumulate")
    torch.cuda.synchronize()


@pytest.mark.parametrize("cin,cout", [(8, 16), (24, 40), (4, 32)])
def test_conv3_backward(cin, cout):
    from paper_2311_16935_amd import unet as U

    announce("conv3 bwd", cin, cout)
    rng = np.random.default_rng(100 + cin)
    shape = (2, 6, 5, 9)
    x = _bf(rng.normal(size=shape + (cin,)))
    W = _bf(rng.normal(size=(27, cin, cout)) / math.sqrt(27 * cin))
    gy = _bf(rng.normal(size=shape + (cout,)))
    rgx, rgW, rgb = O.conv3_backward(x, W, gy)
    xd, wd, gyd = _dev_bf(x), _dev_bf(W), _dev_bf(gy)
    wt = torch.empty((27, cout, cin), dtype=torch.bfloat16, device=DEV)
    U.pu_transpose_taps(wd, wt, 27, cin, cout)
    same = bool(torch.equal(wt.cpu(), wd.cpu().permute(0, 2, 1).contiguous()))
    assert same, 'per-tap transpose differs'
    # data gradient: the layer's [tap][cin][cout] weights are [tap][N = cin][K = cout]
    gx = torch.zeros(shape + (cin,), dtype=torch.float32, device=DEV)
    U.pu_conv(U.tensor(gyd), wd, 27, NEG3, None, U.tensor(gx), shape[1:], y_fp32=True)
    _check(_host(gx), rgx, False, "dgrad")
    npos = math.prod(shape)
    work = torch.zeros(U.pu_wgrad_work_floats(27, cin, cout, npos), dtype=torch.float32, device=DEV)
    dW = torch.zeros((27, cin, cout), dtype=torch.float32, device=DEV)
    db = torch.zeros(cout, dtype=torch.float32, device=DEV)
    U.pu_conv_wgrad(U.tensor(xd), U.tensor(gyd), 27, TAPS3, dW, db, shape[1:], 1, 1, (0, 0, 0), work)
    _check(_host(dW), rgW, False, "wgrad")
    _check(_host(db), rgb, False, "bias grad")
    torch.cuda.synchronize()


def test_wgrad_splits_many_chunks():
    """Enough positions for several position chunks (split-K partials)."""
    from paper_2311_16935_amd import unet as U

    announce("wgrad chunks")
    rng = np.random.default_rng(7)
    shape = (1, 24, 20, 28)
    cin, cout = 16, 24
    x = _bf(rng.normal(size=shape + (cin,)))
    gy = _bf(rng.normal(size=shape + (cout,)))
    _, rgW, rgb = O.conv3_backward(x, np.zeros((27, cin, cout)), gy)
    npos = math.prod(shape)
    work = torch.zeros(U.pu_wgrad_work_floats(27, cin, cout, npos), dtype=torch.float32, device=DEV)
    dW = torch.zeros((27, cin, cout), dtype=torch.float32, device=DEV)
    db = torch.zeros(cout, dtype=torch.float32, device=DEV)
    xd, gyd = _dev_bf(x), _dev_bf(gy)  # descriptors hold raw pointers: keep the tensors alive
    U.pu_conv_wgrad(U.tensor(xd), U.tensor(gyd), 27, TAPS3, dW, db, shape[1:], 1, 1, (0, 0, 0), work)
    _check(_host(dW), rgW, False, "wgrad")
    _check(_host(db), rgb, False, "bias grad")


def test_upconv_forward_backward():
    from paper_2311_16935_amd import unet as U

    announce("upconv")
    rng = np.random.default_rng(11)
    cin, cout = 24, 16
    shape = (2, 3, 2, 4)
    x = _bf(rng.normal(size=shape + (cin,)))
    W = _bf(rng.normal(size=(8, cin, cout)) / math.sqrt(cin))
    fine = (2, 6, 4, 8)
    gy = _bf(rng.normal(size=fine + (cout,)))
    ref = O.upconv(x, W, np.zeros(cout))
    rgx, rgW, _ = O.upconv_backward(x, W, gy)
    xd, wd, gyd = _dev_bf(x), _dev_bf(W), _dev_bf(gy)
    y = torch.zeros(fine + (cout,), dtype=torch.float32, device=DEV)
    wt = torch.empty((8, cout, cin), dtype=torch.bfloat16, device=DEV)
    U.pu_transpose_taps(wd, wt, 8, cin, cout)
    for q, oo in enumerate(UP8):
        U.pu_conv(U.tensor(xd), wt[q], 1, [(0, 0, 0)], None, U.tensor(y), shape[1:], 1, 2, oo, y_fp32=True)
    _check(_host(y), ref, False, "upconv fwd")
    gx = torch.zeros(shape + (cin,), dtype=torch.float32, device=DEV)
    U.pu_conv(U.tensor(gyd), wd, 8, UP8, None, U.tensor(gx), shape[1:], 2, 1, (0, 0, 0), y_fp32=True)
    _check(_host(gx), rgx, False, "upconv dgrad")
    work = torch.zeros(U.pu_wgrad_work_floats(1, cin, cout, math.prod(shape)), dtype=torch.float32, device=DEV)
    dW = torch.zeros((8, cin, cout), dtype=torch.float32, device=DEV)
    for q, oo in enumerate(UP8):
        U.pu_conv_wgrad(U.tensor(xd), U.tensor(gyd), 1, [(0, 0, 0)], dW[q], None, shape[1:], 1, 2, oo, work)
    _check(_host(dW), rgW, False, "upconv wgrad")


def test_pool_relu_head_mse_adam():
    from paper_2311_16935_amd import unet as U

    announce("pool/relu/head/mse/adam")
    rng = np.random.default_rng(12)
    x = _bf(rng.normal(size=(2, 4, 6, 8, 16)))
    xd = _dev_bf(x)
    y = torch.zeros((2, 2, 3, 4, 16), dtype=torch.bfloat16, device=DEV)
    U.pu_pool(U.tensor(xd), U.tensor(y))
    _check(_host(y), O.pool(x), True, "pool")
    gy = _bf(rng.normal(size=(2, 2, 3, 4, 16)))
    gx = torch.from_numpy(np.ones((2, 4, 6, 8, 16), np.float32)).to(torch.bfloat16).to(DEV)
    U.pu_pool_backward(U.tensor(_dev_bf(gy)), U.tensor(gx), True)
    _check(_host(gx), O.pool_backward(gy) + 1.0, True, "pool backward accumulate")
    # relu backward: g zeroed where y <= 0
    g = _bf(rng.normal(size=x.shape))
    gd = _dev_bf(g)
    U.pu_relu_backward(U.tensor(xd), U.tensor(gd))
    assert np.array_equal(_host(gd), np.where(x > 0, g, 0.0))
    # head and masked mse
    w = rng.normal(size=16).astype(np.float32).astype(np.float64)
    b = np.array([0.25])
    ref = O.head(x, w, b[0])
    yd = torch.zeros(x.shape[:4], dtype=torch.float32, device=DEV)
    U.pu_head(U.tensor(xd), _dev_f(w), _dev_f(b), yd)
    _check(_host(yd), ref, False, "head")
    target = rng.normal(size=ref.shape).astype(np.float32).astype(np.float64)
    mask = (rng.uniform(size=ref.shape) > 0.25).astype(np.uint8)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    grad = torch.zeros_like(yd)
    small = torch.zeros(U.HEAD_WORK_FLOATS(16), dtype=torch.float32, device=DEV)
    pred = _host(yd)
    U.pu_mse(yd, _dev_f(target), torch.from_numpy(mask).to(DEV), yd.numel(), loss, grad, small)
    rl, rg = O.mse(pred, target, mask.astype(bool))
    assert float(loss.item()) == pytest.approx(rl, rel=1e-5)
    _check(_host(grad), rg, False, "mse grad")
    gxd = torch.zeros_like(xd)
    gw = torch.zeros(16, dtype=torch.float32, device=DEV)
    gb = torch.zeros(1, dtype=torch.float32, device=DEV)
    U.pu_head_backward(U.tensor(xd), _dev_f(w), grad, U.tensor(gxd), gw, gb, small)
    rgx, rgw, rgb = O.head_backward(x, w, _host(grad))
    _check(_host(gxd), rgx, True, "head dx")
    _check(_host(gw), rgw, False, "head dw")
    assert float(gb.item()) == pytest.approx(rgb, rel=1e-4, abs=1e-6)
    # adam: three steps against the oracle
    n = 1000
    w0 = rng.normal(size=n)
    wd = _dev_f(w0)
    md, vd = torch.zeros_like(wd), torch.zeros_like(wd)
    wb = torch.zeros(n, dtype=torch.bfloat16, device=DEV)
    rw, rm, rv = w0.astype(np.float32).astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        gr = rng.normal(size=n).astype(np.float32).astype(np.float64)
        U.pu_adam(wd, _dev_f(gr), md, vd, wb, n, 1e-2, 0.9, 0.999, 1e-8, step)
        rw, rm, rv = O.adam(rw, gr, rm, rv, 1e-2, 0.9, 0.999, 1e-8, step)
    assert np.abs(_host(wd) - rw).max() <= 1e-6
    assert bool(torch.equal(wb.cpu(), wd.cpu().to(torch.bfloat16))), 'bf16 copy differs'


def test_prepare_input_upsample_and_rms():
    from paper_2311_16935_amd import unet as U

    announce("prepare/upsample/rms")
    rng = np.random.default_rng(13)
    nz, ny, nx, f = 8, 12, 16, 4
    g = [rng.normal(size=(nz, ny, nx)).astype(np.float32).astype(np.float64) for _ in range(3)]
    mask = (rng.uniform(size=(nz, ny, nx)) > 0.2).astype(np.uint8)
    gd = [_dev_f(a) for a in g]
    md = torch.from_numpy(mask).to(DEV)
    out = torch.zeros((1, nz // f, ny // f, nx // f, 4), dtype=torch.bfloat16, device=DEV)
    U.pu_prepare_input(gd[0], gd[1], gd[2], md, (nx, ny, nz), f, 0.5, U.tensor(out))
    ref = O.block_mean([0.5 * a for a in g], mask, f)
    _check(_host(out)[0], ref, True, "prepare_input")
    rms = torch.zeros(1, dtype=torch.float32, device=DEV)
    small = torch.zeros(U.RMS_WORK_FLOATS, dtype=torch.float32, device=DEV)
    U.pu_grad_rms(gd[0], gd[1], gd[2], md, nx * ny * nz, rms, small)
    mb = mask.astype(bool)
    assert float(rms.item()) == pytest.approx(math.sqrt(sum((a[mb] ** 2).sum() for a in g) / mb.sum()), rel=1e-5)
    coarse = rng.normal(size=(nz // f, ny // f, nx // f)).astype(np.float32).astype(np.float64)
    for fp64 in (False, True):
        P = torch.zeros((nz, ny, nx), dtype=torch.float64 if fp64 else torch.float32, device=DEV)
        U.pu_upsample_output(_dev_f(coarse), (nx, ny, nz), f, 3.0, P, fp64)
        _check(_host(P), 3.0 * O.upsample_linear(coarse, f), False, f"upsample fp64={fp64}")
        U.pu_upsample_output(_dev_f(coarse), (nx, ny, nz), f, -1.0, P, fp64, add=True)
        _check(_host(P), 2.0 * O.upsample_linear(coarse, f), False, f"upsample add fp64={fp64}")
    # FP32 coarse-grid means of the gradient components (the coarse solve's input)
    co = [torch.zeros((nz // f, ny // f, nx // f), dtype=torch.float32, device=DEV) for _ in range(3)]
    U.pu_block_mean(gd[0], gd[1], gd[2], md, (nx, ny, nz), f, co[0], co[1], co[2])
    for k in range(3):
        assert np.abs(_host(co[k]) - ref[..., k] / 0.5).max() <= 1e-5 * (1 + np.abs(ref[..., k]).max() / 0.5), k
    # 2-D grid: one plane, no z component
    out2 = torch.zeros((1, 1, ny // f, nx // f, 4), dtype=torch.bfloat16, device=DEV)
    U.pu_prepare_input(gd[0][0], gd[1][0], None, md[0], (nx, ny), f, 1.0, U.tensor(out2))
    ref2 = O.block_mean([g[0][0], g[1][0], np.zeros((ny, nx))], mask[0], f)
    _check(_host(out2)[0, 0], ref2, True, "prepare_input 2d")


# ------------------------------------------------------------ whole network
def _oracle_network(P, x, target, levels, ch, q=lambda a: a):
    """FP64 forward and backward of the U-Net composed from the layer oracle;
    P maps layer name -> (W, b).  q is applied wherever the device stores a
    tensor (activations and their gradients are kept in BF16 there), so the
    comparison isolates the kernels' arithmetic from the storage format.
    Returns loss and name -> (gW, gb)."""
    top = levels - 1
    acts = {}
    h = x
    for l in range(levels):
        a = q(O.conv3(h, *P[f"enc{l}a"], relu=True))
        e = q(O.conv3(a, *P[f"enc{l}b"], relu=True))
        acts[f"in{l}"], acts[f"t{l}"], acts[f"e{l}"] = h, a, e
        if l < top:
            h = q(O.pool(e))
    u = acts[f"e{top}"]
    for l in reversed(range(top)):
        up = q(O.upconv(u, P[f"up{l}"][0], np.zeros(ch[l])))
        cat = np.concatenate([up, acts[f"e{l}"]], axis=-1)
        ua = q(O.conv3(cat, *P[f"dec{l}a"], relu=True))
        ub = q(O.conv3(ua, *P[f"dec{l}b"], relu=True))
        acts[f"u{l}"], acts[f"cat{l}"], acts[f"ua{l}"], acts[f"ub{l}"] = u, cat, ua, ub
        u = ub
    y = O.head(u, P["head"][0][0, :, 0], P["head"][1][0])
    loss, gy = O.mse(y, target, np.ones(y.shape, bool))
    G = {}
    gx, gw, gb = O.head_backward(u, P["head"][0][0, :, 0], gy)
    G["head"] = (gw, np.array([gb]))
    g = q(gx)
    for l in range(top):
        g = g * (acts[f"ub{l}"] > 0)
        gin, gW, gB = O.conv3_backward(acts[f"ua{l}"], P[f"dec{l}b"][0], g)
        G[f"dec{l}b"] = (gW, gB)
        g = q(gin) * (acts[f"ua{l}"] > 0)
        gcat, gW, gB = O.conv3_backward(acts[f"cat{l}"], P[f"dec{l}a"][0], g)
        G[f"dec{l}a"] = (gW, gB)
        gcat = q(gcat)
        acts[f"gskip{l}"] = gcat[..., ch[l]:]
        gu, gW, _ = O.upconv_backward(acts[f"u{l}"], P[f"up{l}"][0], gcat[..., :ch[l]])
        G[f"up{l}"] = (gW, None)
        g = q(gu)
    for l in reversed(range(levels)):
        if l < top:
            g = q(acts[f"gskip{l}"] + O.pool_backward(g))
        g = g * (acts[f"e{l}"] > 0)
        gin, gW, gB = O.conv3_backward(acts[f"t{l}"], P[f"enc{l}b"][0], g)
        G[f"enc{l}b"] = (gW, gB)
        g = q(gin) * (acts[f"t{l}"] > 0)
        gin, gW, gB = O.conv3_backward(acts[f"in{l}"], P[f"enc{l}a"][0], g)
        G[f"enc{l}a"] = (gW, gB)
        g = q(gin)
    return loss, G


def test_network_gradients_match_oracle_composition():
    from paper_2311_16935_amd.warmstart import UNet
    from paper_2311_16935_amd import unet as U

    announce("unet gradients")
    levels, base = 3, 8
    net = UNet(base=base, levels=levels, cin=4, device=DEV, seed=3)
    rng = np.random.default_rng(14)
    res = (8, 8, 12)
    B = net.buffers(1, res)
    x = _bf(rng.normal(size=(1,) + res + (4,)))
    B["x0"].copy_(_dev_bf(x))
    target = rng.normal(size=(1,) + res).astype(np.float32).astype(np.float64)
    P = {}
    master = _host(net.master)
    wb = _host(net.wb)
    for name, L in net.layers.items():
        src = master if L.kind == "head" else wb
        W = src[L.off_w:L.off_w + L.wsize].reshape(L.taps, L.cin, L.cout)
        b = master[L.off_b:L.off_b + L.cout] if L.off_b >= 0 else None
        P[name] = (W, b)
    rloss, RG = _oracle_network(P, x, target, levels, net.ch, q=_bf)
    net.forward(B)
    U.pu_mse(B["y"], _dev_f(target), None, B["y"].numel(), net.loss, B["gy"], net.small)
    net.backward(B)
    torch.cuda.synchronize()
    assert float(net.loss.item()) == pytest.approx(rloss, rel=1e-3)
    grad = _host(net.grad)
    errs = {}
    for name, L in net.layers.items():
        gW = grad[L.off_w:L.off_w + L.wsize].reshape(L.taps, L.cin, L.cout)
        rW, rb = RG[name]
        rW = np.asarray(rW).reshape(gW.shape)
        errs[name] = np.linalg.norm(gW - rW) / np.linalg.norm(rW)
        if rb is not None:
            gb = grad[L.off_b:L.off_b + L.cout]
            errs[name + ".b"] = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
    print({k: f"{v:.2e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= 1e-2}
    assert not bad, f"relative L2 gradient errors above 1e-2: {bad}"


def test_training_reduces_loss_on_a_fixed_batch():
    from paper_2311_16935_amd.warmstart import UNet

    announce("unet overfit")
    net = UNet(base=8, levels=3, cin=4, device=DEV, seed=5)
    rng = np.random.default_rng(15)
    res = (8, 8, 8)
    B = net.buffers(2, res)
    B["x0"].copy_(_dev_bf(rng.normal(size=(2,) + res + (4,))))
    zz = np.linspace(-1, 1, 8)
    target = _dev_f(np.broadcast_to(np.sin(3 * zz)[None, :, None, None], (2,) + res).copy())
    first = None
    for _ in range(60):
        net.train_step(B, target, 3e-3)
        if first is None:
            first = float(net.loss.item())
    last = float(net.loss.item())
    assert last < 0.3 * first, (first, last)
