"""MI355X solver for matrix-based omnidirectional pressure integration.

Thin ctypes binding of ``libpi.so`` (see ``include/pi.h``).  Functions carry
the C names (``pi_plan``, ``pi_solve``, ``pi_solve_batched``, ``pi_source``,
``pi_apply`` ...) and only marshal arguments: torch tensors supply device
memory and the current stream; every step of the solve runs in the library's
HIP kernels.  There is no CPU fallback: if the library is missing or cannot
be loaded, importing this package raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch  # loads the HIP runtime that libpi then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpi.so")

PI_OK = 0
PI_ERR_INVALID_ARG = 1
PI_ERR_OOM = 2
PI_ERR_NONFINITE = 3
PI_ERR_NOT_CONVERGED = 4
PI_ERR_DIVERGED = 5
PI_ERR_DEVICE = 6
PI_ERR_TOO_LARGE = 7
PI_NOALLOC_MAX_INSTANCES = 1024
PI_NOALLOC_MAX_PARTIALS = 262144
PI_NOALLOC_MAX_TABLE = 524288

PI_FP32 = 0x0
PI_FP64 = 0x1
PI_INNER_CG = 0x0
PI_INNER_BICGSTAB = 0x2
PI_FIXED_POINT_CG = 0x4
PI_CELL_CENTERED = 0x8
PI_WARM_START = 0x1
PI_ASYNC = 0x2
PI_OP_M, PI_OP_N, PI_OP_L = 0, 1, 2


class PiInfo(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int64),
        ("inner_iters_total", ctypes.c_int64),
        ("eps_R", ctypes.c_double),
        ("eps_P", ctypes.c_double),
        ("ms", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("components", ctypes.c_int32),
        ("worklist_rebuilds", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2311_16935_amd/build.py` "
                          "(or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.pi_plan.argtypes = [ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.c_void_p, u32,
                            ctypes.POINTER(vp)]
    lib.pi_plan.restype = ctypes.c_int
    lib.pi_plan_destroy.argtypes = [vp]
    lib.pi_plan_destroy.restype = None
    lib.pi_workspace_bytes.argtypes = [vp]
    lib.pi_workspace_bytes.restype = ctypes.c_size_t
    lib.pi_set_inner_iters.argtypes = [vp, ctypes.c_int32]
    lib.pi_set_inner_iters.restype = ctypes.c_int
    lib.pi_solve.argtypes = [vp, vp, vp, vp, vp, dbl, i64, u32, ctypes.POINTER(PiInfo), vp]
    lib.pi_solve.restype = ctypes.c_int
    lib.pi_solve_batched.argtypes = [i64, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(dbl), i64, u32,
                                     ctypes.POINTER(PiInfo), vp]
    lib.pi_solve_batched.restype = ctypes.c_int
    lib.pi_solve_batched_noalloc.argtypes = lib.pi_solve_batched.argtypes
    lib.pi_solve_batched_noalloc.restype = ctypes.c_int
    lib.pi_last_info.argtypes = [vp, ctypes.POINTER(PiInfo)]
    lib.pi_last_info.restype = ctypes.c_int
    lib.pi_source.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.pi_source.restype = ctypes.c_int
    lib.pi_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.pi_apply.restype = ctypes.c_int
    lib.pi_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.pi_set_tile.restype = ctypes.c_int
    lib.pi_get_tile.argtypes = [vp]
    lib.pi_get_tile.restype = ctypes.c_int32
    lib.pi_get_lane_cells.argtypes = [vp]
    lib.pi_get_lane_cells.restype = ctypes.c_int32
    lib.pi_get_cg_recompute.argtypes = [vp]
    lib.pi_get_cg_recompute.restype = ctypes.c_int32
    lib.pi_time_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(dbl), vp]
    lib.pi_time_kernel.restype = ctypes.c_int
    lib.pi_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp]
    lib.pi_autotune.restype = ctypes.c_int
    lib.pi_status_string.argtypes = [ctypes.c_int]
    lib.pi_status_string.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTED = ("pi_plan", "pi_plan_destroy", "pi_workspace_bytes", "pi_set_inner_iters", "pi_set_tile",
            "pi_get_tile", "pi_get_lane_cells", "pi_get_cg_recompute", "pi_solve", "pi_last_info",
            "pi_solve_batched", "pi_solve_batched_noalloc", "pi_source", "pi_apply", "pi_time_kernel", "pi_autotune", "pi_status_string")

PI_K_OUTER, PI_K_INNER = 0, 1


class PiError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {pi_status_string(status)} (status {status})")


def pi_status_string(status: int) -> str:
    return lib.pi_status_string(int(status)).decode()


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def pi_plan(ndim: int, dims: Sequence[int], spacing: Sequence[float], mask=None, flags: int = 0) -> ctypes.c_void_p:
    d = (ctypes.c_int64 * 3)(*(list(int(v) for v in dims) + [1] * (3 - len(dims))))
    s = (ctypes.c_double * 3)(*(list(float(v) for v in spacing) + [1.0] * (3 - len(spacing))))
    mptr = None
    keep = None
    if mask is not None:
        m = mask.detach().to("cpu", torch.uint8).contiguous() if isinstance(mask, torch.Tensor) else \
            torch.as_tensor(mask, dtype=torch.uint8).contiguous()
        keep = m
        mptr = ctypes.c_void_p(m.data_ptr())
    out = ctypes.c_void_p()
    rc = lib.pi_plan(int(ndim), d, s, mptr, ctypes.c_uint32(flags), ctypes.byref(out))
    del keep
    if rc != PI_OK:
        raise PiError(rc, "pi_plan")
    return out


def pi_plan_destroy(plan) -> None:
    lib.pi_plan_destroy(plan)


def pi_workspace_bytes(plan) -> int:
    return int(lib.pi_workspace_bytes(plan))


def pi_set_inner_iters(plan, iters: int) -> None:
    rc = lib.pi_set_inner_iters(plan, int(iters))
    if rc != PI_OK:
        raise PiError(rc, "pi_set_inner_iters")


def pi_set_tile(plan, mseg: int, lane_cells: int = 0) -> None:
    rc = lib.pi_set_tile(plan, int(mseg), int(lane_cells))
    if rc != PI_OK:
        raise PiError(rc, "pi_set_tile")


def pi_get_tile(plan) -> int:
    return int(lib.pi_get_tile(plan))


def pi_get_lane_cells(plan) -> int:
    return int(lib.pi_get_lane_cells(plan))


def pi_get_cg_recompute(plan) -> int:
    return int(lib.pi_get_cg_recompute(plan))


def pi_solve(plan, gx, gy, gz, P, tol, max_iter, flags=0, stream=None):
    info = PiInfo()
    rc = lib.pi_solve(plan, _ptr(gx), _ptr(gy), _ptr(gz), _ptr(P), float(tol), int(max_iter),
                      ctypes.c_uint32(flags), ctypes.byref(info), _stream(stream))
    return rc, info


def _batched(fn, plans, gx, gy, gz, P, tol, max_iter, flags, stream):
    n = len(plans)
    vp = ctypes.c_void_p
    arr = lambda xs: (vp * n)(*[None if x is None else x.data_ptr() for x in xs])  # noqa: E731
    infos = (PiInfo * n)()
    rc = fn(n, (vp * n)(*[p.value for p in plans]), arr(gx), arr(gy), arr(gz) if gz is not None else None, arr(P),
            (ctypes.c_double * n)(*tol), int(max_iter), ctypes.c_uint32(flags), infos, _stream(stream))
    return rc, list(infos)


def pi_last_info(plan):
    info = PiInfo()
    rc = lib.pi_last_info(plan, ctypes.byref(info))
    return rc, info


def pi_solve_batched(plans, gx, gy, gz, P, tol, max_iter, flags=0, stream=None):
    return _batched(lib.pi_solve_batched, plans, gx, gy, gz, P, tol, max_iter, flags, stream)


def pi_solve_batched_noalloc(plans, gx, gy, gz, P, tol, max_iter, flags=0, stream=None):
    return _batched(lib.pi_solve_batched_noalloc, plans, gx, gy, gz, P, tol, max_iter, flags, stream)


def pi_source(plan, gx, gy, gz, S, stream=None) -> int:
    return lib.pi_source(plan, _ptr(gx), _ptr(gy), _ptr(gz), _ptr(S), _stream(stream))


def pi_apply(plan, op, x, y, stream=None) -> int:
    return lib.pi_apply(plan, int(op), _ptr(x), _ptr(y), _stream(stream))


def pi_time_kernel(plan, kernel, reps, stream=None) -> float:
    ms = ctypes.c_double()
    rc = lib.pi_time_kernel(plan, int(kernel), int(reps), ctypes.byref(ms), _stream(stream))
    if rc != PI_OK:
        raise PiError(rc, "pi_time_kernel")
    return ms.value


def pi_autotune(plan, reps=5, stream=None) -> int:
    m = ctypes.c_int32()
    rc = lib.pi_autotune(plan, int(reps), ctypes.byref(m), _stream(stream))
    if rc != PI_OK:
        raise PiError(rc, "pi_autotune")
    return m.value


# ---------------------------------------------------------------------------
# convenience layer over the same calls
# ---------------------------------------------------------------------------
@dataclass
class SolveResult:
    P: torch.Tensor
    status: int
    info: dict


class Plan:
    """A planned grid: ``dims`` = (nx, ny[, nz]); tensors are in storage
    order, i.e. shaped (ny, nx) or (nz, ny, nx)."""

    def __init__(self, dims, spacing, mask=None, fp64=False, bicgstab=False, inner_iters=None, fixed_point=False,
                 cell_centered=False):
        self.dims = tuple(int(v) for v in dims)
        self.ndim = len(self.dims)
        self.spacing = tuple(float(v) for v in spacing)
        self.fp64 = bool(fp64)
        self.dtype = torch.float64 if fp64 else torch.float32
        flags = (PI_FP64 if fp64 else PI_FP32) | (PI_INNER_BICGSTAB if bicgstab else PI_INNER_CG)
        if fixed_point:
            flags |= PI_FIXED_POINT_CG
        if cell_centered:
            flags |= PI_CELL_CENTERED
        self.handle = pi_plan(self.ndim, self.dims, self.spacing, mask, flags)
        if inner_iters is not None:
            pi_set_inner_iters(self.handle, inner_iters)

    @property
    def shape(self):
        return tuple(reversed(self.dims))

    @property
    def workspace_bytes(self):
        return pi_workspace_bytes(self.handle)

    def set_inner_iters(self, k):
        pi_set_inner_iters(self.handle, k)

    def autotune(self, reps=5, stream=None):
        """Pick and set the fastest tile for this grid (cached per shape)."""
        return pi_autotune(self.handle, reps, stream)

    def _check(self, t, name):
        if t is None:
            raise ValueError(f"{name} is required")
        if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor of shape {self.shape}")

    def solve_async(self, grads, P, tol=1e-6, max_iter=100000, warm_start=False, stream=None):
        """Enqueue the whole solve on ``stream`` (PI_ASYNC); after the stream
        has completed, ``last_info()`` gives its status and info."""
        gz = grads[2] if self.ndim == 3 else None
        for i, g in enumerate(grads[: self.ndim]):
            self._check(g, f"grad[{i}]")
        self._check(P, "P")
        flags = PI_ASYNC | (PI_WARM_START if warm_start else 0)
        rc, _ = pi_solve(self.handle, grads[0], grads[1], gz, P, tol, max_iter, flags, stream)
        if rc != PI_OK:
            raise PiError(rc, "pi_solve (async)")
        return P

    def last_info(self):
        rc, info = pi_last_info(self.handle)
        return rc, info.as_dict()

    def solve(self, grads, P=None, tol=1e-6, max_iter=10**7, warm_start=False, stream=None, check=True):
        gx, gy = grads[0], grads[1]
        gz = grads[2] if self.ndim == 3 else None
        for i, g in enumerate(grads[: self.ndim]):
            self._check(g, f"grad[{i}]")
        if P is None:
            if warm_start:
                raise ValueError("warm_start needs P")
            P = torch.empty(self.shape, dtype=self.dtype, device=gx.device)
        self._check(P, "P")
        rc, info = pi_solve(self.handle, gx, gy, gz, P, tol, max_iter, PI_WARM_START if warm_start else 0, stream)
        if check and rc not in (PI_OK, PI_ERR_NOT_CONVERGED):
            raise PiError(rc, "pi_solve")
        return SolveResult(P, rc, info.as_dict())

    def source(self, grads, out=None, stream=None):
        gz = grads[2] if self.ndim == 3 else None
        for i, g in enumerate(grads[: self.ndim]):
            self._check(g, f"grad[{i}]")
        out = torch.empty(self.shape, dtype=self.dtype, device=grads[0].device) if out is None else out
        self._check(out, "S")
        rc = pi_source(self.handle, grads[0], grads[1], gz, out, stream)
        if rc != PI_OK:
            raise PiError(rc, "pi_source")
        return out

    def apply(self, op, x, out=None, stream=None):
        self._check(x, "x")
        out = torch.empty_like(x) if out is None else out
        self._check(out, "y")
        rc = pi_apply(self.handle, op, x, out, stream)
        if rc != PI_OK:
            raise PiError(rc, "pi_apply")
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            pi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(plans, grads_list, P_list=None, tol=1e-6, max_iter=10**7, warm_start=False, stream=None,
                  check=True, noalloc=False):
    """One batched solve over ``plans`` (all of one precision); with
    ``noalloc`` through pi_solve_batched_noalloc (no device allocation)."""
    n = len(plans)
    if P_list is None:
        P_list = [torch.empty(p.shape, dtype=p.dtype, device=g[0].device) for p, g in zip(plans, grads_list)]
    for p, g, P in zip(plans, grads_list, P_list):
        for i, t in enumerate(g[: p.ndim]):
            p._check(t, f"grad[{i}]")
        p._check(P, "P")
    tols = [float(tol)] * n if not isinstance(tol, (list, tuple)) else [float(t) for t in tol]
    gz = [g[2] if p.ndim == 3 else None for p, g in zip(plans, grads_list)]
    fn = pi_solve_batched_noalloc if noalloc else pi_solve_batched
    rc, infos = fn([p.handle for p in plans], [g[0] for g in grads_list], [g[1] for g in grads_list], gz, P_list,
                   tols, max_iter, PI_WARM_START if warm_start else 0, stream)
    if check and rc not in (PI_OK, PI_ERR_NOT_CONVERGED):
        raise PiError(rc, fn.__name__)
    return rc, P_list, [i.as_dict() for i in infos]
