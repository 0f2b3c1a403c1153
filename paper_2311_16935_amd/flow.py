"""ctypes binding of the velocity -> source stage (``include/pi_flow.h``).

Same names as the C entry points; velocity, stress and output fields are
FP32 torch tensors on the GPU in the solver's storage order.  The arithmetic
runs in ``libpi.so``.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import PI_OK, PiError, _stream, lib

PI_FLOW_NS, PI_FLOW_RANS, PI_FLOW_COMPRESSIBLE = 0, 1, 2
EXPORTED = ("pi_flow_source",)


class PiFlowParams(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("gas_R", ctypes.c_double), ("gamma", ctypes.c_double), ("T_inf", ctypes.c_double),
                ("M_inf", ctypes.c_double), ("V_inf", ctypes.c_double)]


_P = ctypes.POINTER(ctypes.c_void_p)
lib.pi_flow_source.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                               ctypes.c_int, _P, _P, _P, _P, ctypes.POINTER(PiFlowParams), _P, ctypes.c_void_p]
lib.pi_flow_source.restype = ctypes.c_int


def _ptrs(ts: Optional[Sequence[torch.Tensor]]):
    if ts is None:
        return None
    for t in ts:
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("flow fields are contiguous float32 CUDA tensors")
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def pi_flow_source(model, u, spacing, out=None, u_prev=None, u_next=None, R=None, rho=1.0, mu=0.0, dt=0.0,
                   gas_R=287.0, gamma=1.4, T_inf=1.0, M_inf=0.0, V_inf=1.0, stream=None):
    """Source field from velocity; u is a list of ndim tensors shaped like the
    grid in storage order ((ny, nx) or (nz, ny, nx)).  Returns the list of f
    components."""
    nd = len(u)
    shape = tuple(u[0].shape)
    dims = (ctypes.c_int64 * 3)(*(list(reversed(shape)) + [1] * (3 - nd)))
    sp = (ctypes.c_double * 3)(*(list(float(v) for v in spacing) + [1.0] * (3 - nd)))
    if out is None:
        out = [torch.empty_like(u[0]) for _ in range(nd)]
    prm = PiFlowParams(rho, mu, dt, gas_R, gamma, T_inf, M_inf, V_inf)
    rc = lib.pi_flow_source(nd, dims, sp, int(model), _ptrs(u), _ptrs(u_prev), _ptrs(u_next), _ptrs(R),
                            ctypes.byref(prm), _ptrs(out), _stream(stream))
    if rc != PI_OK:
        raise PiError(rc, "pi_flow_source")
    return out
