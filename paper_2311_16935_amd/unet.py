"""ctypes binding of the warm-start network's layer calls (``include/pi_unet.h``).

Same names as the C entry points; arguments are torch tensors (device memory)
and the current stream.  Every layer's arithmetic runs in ``libpi.so``.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import PI_OK, PiError, _stream, lib

EXPORTED = ("pu_conv", "pu_wgrad_work_floats", "pu_conv_wgrad", "pu_transpose_taps", "pu_relu_backward",
            "pu_pool", "pu_pool_backward", "pu_head", "pu_head_backward", "pu_mse", "pu_adam",
            "pu_prepare_input", "pu_block_mean", "pu_upsample_output", "pu_grad_rms")

# FP32 scratch sizes the element-wise reductions need (see the header)
HEAD_WORK_FLOATS = lambda c: 1025 * (c + 1)  # noqa: E731
MSE_WORK_FLOATS = 2049
RMS_WORK_FLOATS = 1025


class PuTensor(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("n", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32),
                ("w", ctypes.c_int32), ("c", ctypes.c_int32), ("ld", ctypes.c_int32), ("off", ctypes.c_int32)]


def _sig():
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    T = ctypes.POINTER(PuTensor)
    I3 = ctypes.POINTER(ctypes.c_int32)
    L3 = ctypes.POINTER(ctypes.c_int64)
    s = {
        "pu_conv": [T, vp, i32, vp, vp, T, i32, i32, i32, i32, i32, I3, i32, i32, i32, vp],
        "pu_wgrad_work_floats": [i32, i32, i32, i64],
        "pu_conv_wgrad": [T, T, i32, vp, vp, vp, i32, i32, i32, i32, i32, I3, vp, vp],
        "pu_transpose_taps": [vp, vp, i32, i32, i32, vp],
        "pu_relu_backward": [T, T, vp],
        "pu_pool": [T, T, vp],
        "pu_pool_backward": [T, T, i32, vp],
        "pu_head": [T, vp, vp, vp, vp],
        "pu_head_backward": [T, vp, vp, T, vp, vp, vp, vp],
        "pu_mse": [vp, vp, vp, i64, vp, vp, vp, vp],
        "pu_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
        "pu_prepare_input": [vp, vp, vp, vp, L3, i32, f32, T, vp],
        "pu_block_mean": [vp, vp, vp, vp, L3, i32, vp, vp, vp, vp],
        "pu_upsample_output": [vp, L3, i32, f32, vp, i32, vp],
        "pu_grad_rms": [vp, vp, vp, vp, i64, vp, vp, vp],
    }
    for name, args in s.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_size_t if name == "pu_wgrad_work_floats" else ctypes.c_int


_sig()


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ok(rc, where):
    if rc != PI_OK:
        raise PiError(rc, where)


def tensor(t: torch.Tensor, off: int = 0, c: Optional[int] = None) -> PuTensor:
    """Descriptor of channels [off, off + c) of a contiguous [n, d, h, w, ld] tensor."""
    if t.dim() != 5 or not t.is_contiguous():
        raise ValueError("layer tensors are contiguous [n, d, h, w, channels]")
    n, d, h, w, ld = t.shape
    c = ld - off if c is None else c
    return PuTensor(t.data_ptr(), n, d, h, w, c, ld, off)


def _i3(v: Sequence[int]):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def _offs(offs) -> torch.Tensor:
    return torch.as_tensor(offs, dtype=torch.int8).reshape(-1).contiguous()


def pu_conv(x: PuTensor, w, taps, offs, bias, y: PuTensor, m, sin=1, sout=1, oo=(0, 0, 0), relu=False,
            y_fp32=False, accumulate=False, stream=None):
    o = _offs(offs)
    _ok(lib.pu_conv(ctypes.byref(x), _p(w), int(taps), ctypes.c_void_p(o.data_ptr()), _p(bias), ctypes.byref(y),
                    int(m[0]), int(m[1]), int(m[2]), int(sin), int(sout), _i3(oo), int(relu), int(y_fp32),
                    int(accumulate), _stream(stream)), "pu_conv")


def pu_wgrad_work_floats(taps, cin, cout, positions) -> int:
    return int(lib.pu_wgrad_work_floats(int(taps), int(cin), int(cout), int(positions)))


def pu_conv_wgrad(x: PuTensor, gy: PuTensor, taps, offs, dw, db, m, sin, sout, oo, work, stream=None):
    o = _offs(offs)
    _ok(lib.pu_conv_wgrad(ctypes.byref(x), ctypes.byref(gy), int(taps), ctypes.c_void_p(o.data_ptr()), _p(dw),
                          _p(db), int(m[0]), int(m[1]), int(m[2]), int(sin), int(sout), _i3(oo), _p(work),
                          _stream(stream)), "pu_conv_wgrad")


def pu_transpose_taps(w, wt, taps, cin, cout, stream=None):
    _ok(lib.pu_transpose_taps(_p(w), _p(wt), int(taps), int(cin), int(cout), _stream(stream)), "pu_transpose_taps")


def pu_relu_backward(y: PuTensor, g: PuTensor, stream=None):
    _ok(lib.pu_relu_backward(ctypes.byref(y), ctypes.byref(g), _stream(stream)), "pu_relu_backward")


def pu_pool(x: PuTensor, y: PuTensor, stream=None):
    _ok(lib.pu_pool(ctypes.byref(x), ctypes.byref(y), _stream(stream)), "pu_pool")


def pu_pool_backward(gy: PuTensor, gx: PuTensor, accumulate=False, stream=None):
    _ok(lib.pu_pool_backward(ctypes.byref(gy), ctypes.byref(gx), int(accumulate), _stream(stream)),
        "pu_pool_backward")


def pu_head(x: PuTensor, w, b, y, stream=None):
    _ok(lib.pu_head(ctypes.byref(x), _p(w), _p(b), _p(y), _stream(stream)), "pu_head")


def pu_head_backward(x: PuTensor, w, gy, gx: PuTensor, gw, gb, work, stream=None):
    _ok(lib.pu_head_backward(ctypes.byref(x), _p(w), _p(gy), ctypes.byref(gx), _p(gw), _p(gb), _p(work),
                             _stream(stream)), "pu_head_backward")


def pu_mse(pred, target, mask, count, loss, grad, work, stream=None):
    _ok(lib.pu_mse(_p(pred), _p(target), _p(mask), int(count), _p(loss), _p(grad), _p(work), _stream(stream)),
        "pu_mse")


def pu_adam(w, g, m, v, wb, count, lr, beta1, beta2, eps, step, stream=None):
    _ok(lib.pu_adam(_p(w), _p(g), _p(m), _p(v), _p(wb), int(count), float(lr), float(beta1), float(beta2),
                    float(eps), int(step), _stream(stream)), "pu_adam")


def pu_prepare_input(gx, gy, gz, mask, dims, factor, scale, out: PuTensor, stream=None):
    d = (ctypes.c_int64 * 3)(*(list(int(v) for v in dims) + [1] * (3 - len(dims))))
    _ok(lib.pu_prepare_input(_p(gx), _p(gy), _p(gz), _p(mask), d, int(factor), float(scale), ctypes.byref(out),
                             _stream(stream)), "pu_prepare_input")


def pu_block_mean(gx, gy, gz, mask, dims, factor, ox, oy, oz, stream=None):
    d = (ctypes.c_int64 * 3)(*(list(int(v) for v in dims) + [1] * (3 - len(dims))))
    _ok(lib.pu_block_mean(_p(gx), _p(gy), _p(gz), _p(mask), d, int(factor), _p(ox), _p(oy), _p(oz),
                          _stream(stream)), "pu_block_mean")


PU_OUT_FP64, PU_OUT_ADD = 0x1, 0x2


def pu_upsample_output(coarse, dims, factor, scale, P, fp64=False, stream=None, add=False):
    d = (ctypes.c_int64 * 3)(*(list(int(v) for v in dims) + [1] * (3 - len(dims))))
    flags = (PU_OUT_FP64 if fp64 else 0) | (PU_OUT_ADD if add else 0)
    _ok(lib.pu_upsample_output(_p(coarse), d, int(factor), float(scale), _p(P), flags, _stream(stream)),
        "pu_upsample_output")


def pu_grad_rms(gx, gy, gz, mask, count, rms, work, stream=None):
    _ok(lib.pu_grad_rms(_p(gx), _p(gy), _p(gz), _p(mask), int(count), _p(rms), _p(work), _stream(stream)),
        "pu_grad_rms")
