"""Learned warm start: a 3-D convolutional U-Net that maps a pressure-gradient
field to an initial pressure guess {P^0} for Algorithm 1.

The paper starts Algorithm 1 from {P^0} = 0; its convergence study (Sections
"Effect of Pressure Magnitude at the Boundaries" and "Wall-clock Time
Convergence") shows that the iteration count depends on how far the starting
field is from the answer.  The network supplies a better start; the plain
solver then finishes from it, so the converged field is the method's own and
the network can only change the iteration count.

Architecture (4 levels, base width 32): per level two 3x3x3 convolutions with
ReLU (32/64/128/256 channels), 2x2x2 average pooling on the way down, 2x2x2
stride-2 transposed convolutions on the way up, channel concatenation of the
encoder features, and a 1x1x1 head.  Activations are channels-last BF16,
accumulation FP32, master weights FP32 with Adam.  Every layer, its gradient
and the optimizer step run in the library's kernels (``include/pi_unet.h``);
this module owns the buffers and the order of the calls.

Scaling: the input is the gradient divided by its RMS over the data cells, on
a grid coarsened by ``factor``; the output is the pressure in units of
RMS * (network cell size), so a network trained on one grid size serves
another grid over the same physical domain at the same network resolution.
"""

from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass

import torch

from . import Plan, solve_batched
from . import unet as U

TAPS3 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
NEG3 = [(-dz, -dy, -dx) for (dz, dy, dx) in TAPS3]
UP8 = [(q >> 2, (q >> 1) & 1, q & 1) for q in range(8)]
ZERO1 = [(0, 0, 0)]
BF16 = torch.bfloat16


@dataclass
class Layer:
    name: str
    kind: str  # "conv", "up" or "head"
    cin: int
    cout: int
    taps: int
    off_w: int
    off_b: int  # -1: no bias

    @property
    def wsize(self):
        return self.taps * self.cin * self.cout


def _align(n, a=64):
    return (n + a - 1) // a * a


class UNet:
    @staticmethod
    def layout(base=32, levels=4, cin=4):
        """Layers in call order and their slices of the flat parameter buffer
        (every slice starts on a 64-element boundary); returns (layers, size)."""
        ch = [base << l for l in range(levels)]
        layers = {}
        off = 0

        def add(name, kind, ci, co, taps, bias=True):
            nonlocal off
            ow = off
            off = _align(off + taps * ci * co)
            ob = -1
            if bias:
                ob = off
                off = _align(off + co)
            layers[name] = Layer(name, kind, ci, co, taps, ow, ob)

        for l in range(levels):
            add(f"enc{l}a", "conv", cin if l == 0 else ch[l - 1], ch[l], 27)
            add(f"enc{l}b", "conv", ch[l], ch[l], 27)
        for l in reversed(range(levels - 1)):
            add(f"up{l}", "up", ch[l + 1], ch[l], 8, bias=False)
            add(f"dec{l}a", "conv", 2 * ch[l], ch[l], 27)
            add(f"dec{l}b", "conv", ch[l], ch[l], 27)
        add("head", "head", ch[0], 1, 1)
        return layers, off

    def __init__(self, base=32, levels=4, cin=4, device="cuda:0", seed=0):
        self.base, self.levels, self.cin, self.device = base, levels, cin, torch.device(device)
        self.ch = [base << l for l in range(levels)]
        self.layers, off = self.layout(base, levels, cin)
        self.nparams = off
        dev = self.device
        self.master = torch.zeros(off, dtype=torch.float32, device=dev)
        self._init(seed)
        self.wb = self.master.to(BF16)
        self.wt = torch.zeros(off, dtype=BF16, device=dev)
        self.grad = torch.zeros(off, dtype=torch.float32, device=dev)
        self.m = torch.zeros(off, dtype=torch.float32, device=dev)
        self.v = torch.zeros(off, dtype=torch.float32, device=dev)
        self.step_count = 0
        self._refresh_transposed()
        self._bufs = {}
        self.small = torch.zeros(max(U.HEAD_WORK_FLOATS(self.ch[0]), U.MSE_WORK_FLOATS, U.RMS_WORK_FLOATS),
                                 dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)

    # ------------------------------------------------------------------ params
    def _init(self, seed):
        """He-normal weights, zero biases (drawn on the host so the start does
        not depend on the device)."""
        g = torch.Generator().manual_seed(seed)
        host = torch.zeros(self.nparams, dtype=torch.float32)
        for L in self.layers.values():
            fan_in = L.taps * L.cin if L.kind != "up" else L.cin
            std = math.sqrt(2.0 / fan_in) if L.kind != "head" else math.sqrt(1.0 / L.cin)
            host[L.off_w:L.off_w + L.wsize] = torch.randn(L.wsize, generator=g) * std
        self.master.copy_(host)

    def w(self, name, buf=None):
        L = self.layers[name]
        b = self.wb if buf is None else buf
        return b[L.off_w:L.off_w + L.wsize]

    def b(self, name, buf=None):
        L = self.layers[name]
        b = self.master if buf is None else buf
        return None if L.off_b < 0 else b[L.off_b:L.off_b + L.cout]

    def _refresh_transposed(self):
        for L in self.layers.values():
            if L.kind in ("conv", "up"):
                U.pu_transpose_taps(self.w(L.name), self.w(L.name, self.wt), L.taps, L.cin, L.cout)

    def state_dict(self):
        meta = {"base": self.base, "levels": self.levels, "cin": self.cin, "step": self.step_count}
        return {"master_bf16": self.master.to(BF16).cpu()}, meta

    def load(self, tensors, meta):
        if (meta["base"], meta["levels"], meta["cin"]) != (self.base, self.levels, self.cin):
            raise ValueError("weights were saved for another architecture")
        self.master.copy_(tensors["master_bf16"].to(self.device, torch.float32))
        self.wb.copy_(self.master.to(BF16))
        self._refresh_transposed()

    def save(self, path, extra=None):
        from safetensors.torch import save_file

        t, meta = self.state_dict()
        meta.update(extra or {})
        save_file(t, path, metadata={"unet": json.dumps(meta)})

    @classmethod
    def from_file(cls, path, device="cuda:0"):
        from safetensors import safe_open

        with safe_open(path, framework="pt") as f:
            meta = json.loads(f.metadata()["unet"])
            t = {k: f.get_tensor(k) for k in f.keys()}
        net = cls(base=meta["base"], levels=meta["levels"], cin=meta["cin"], device=device)
        net.load(t, meta)
        net.meta = meta
        return net

    # ----------------------------------------------------------------- buffers
    def buffers(self, n, res):
        """Activation and gradient buffers for batch n at grid res = (D, H, W)."""
        key = (n, tuple(res))
        if key in self._bufs:
            return self._bufs[key]
        D, H, W = res
        f = 1 << (self.levels - 1)
        if D % f or H % f or W % f:
            raise ValueError(f"network grid {res} must be divisible by {f}")
        dev = self.device
        R = [(D >> l, H >> l, W >> l) for l in range(self.levels)]
        z = lambda r, c: torch.zeros((n,) + r + (c,), dtype=BF16, device=dev)  # noqa: E731
        B = {"R": R, "n": n}
        B["x0"] = z(R[0], self.cin)
        for l in range(self.levels):
            B[f"t{l}"], B[f"gt{l}"] = z(R[l], self.ch[l]), z(R[l], self.ch[l])
            if l < self.levels - 1:
                B[f"cat{l}"], B[f"gcat{l}"] = z(R[l], 2 * self.ch[l]), z(R[l], 2 * self.ch[l])
                B[f"ua{l}"], B[f"gua{l}"] = z(R[l], self.ch[l]), z(R[l], self.ch[l])
                B[f"ub{l}"], B[f"gub{l}"] = z(R[l], self.ch[l]), z(R[l], self.ch[l])
            if l > 0:
                B[f"p{l}"], B[f"gp{l}"] = z(R[l], self.ch[l - 1]), z(R[l], self.ch[l - 1])
        top = self.levels - 1
        B["bot"], B["gbot"] = z(R[top], self.ch[top]), z(R[top], self.ch[top])
        B["y"] = torch.zeros((n,) + R[0], dtype=torch.float32, device=dev)
        B["gy"] = torch.zeros_like(B["y"])
        work = 0
        for L in self.layers.values():
            if L.kind == "conv":
                lvl = int(L.name[3])
                work = max(work, U.pu_wgrad_work_floats(L.taps, L.cin, L.cout, n * math.prod(R[lvl])))
            elif L.kind == "up":
                lvl = int(L.name[2]) + 1
                work = max(work, U.pu_wgrad_work_floats(1, L.cin, L.cout, n * math.prod(R[lvl])))
        B["work"] = torch.zeros(work, dtype=torch.float32, device=dev)
        self._bufs[key] = B
        return B

    def release(self):
        self._bufs.clear()

    # ------------------------------------------------------------------ layers
    def _conv(self, name, x, y, m, relu=True, stream=None):
        U.pu_conv(x, self.w(name, self.wt), 27, TAPS3, self.b(name), y, m, 1, 1, (0, 0, 0), relu, False, False,
                  stream)

    def _conv_back(self, name, x, g, gx, m, B, stream=None):
        """g holds dL/d(pre-activation) of layer `name` with input x: writes its
        weight and bias gradients and, if gx is given, dL/dx."""
        L = self.layers[name]
        U.pu_conv_wgrad(x, g, 27, TAPS3, self.w(name, self.grad), self.b(name, self.grad), m, 1, 1, (0, 0, 0),
                        B["work"], stream)
        if gx is not None:
            U.pu_conv(g, self.w(name), 27, NEG3, None, gx, m, 1, 1, (0, 0, 0), False, False, False, stream)

    def forward(self, B, stream=None):
        T = U.tensor
        R, top = B["R"], self.levels - 1
        for l in range(self.levels):
            src = T(B["x0"]) if l == 0 else T(B[f"p{l}"])
            self._conv(f"enc{l}a", src, T(B[f"t{l}"]), R[l], stream=stream)
            dst = T(B[f"cat{l}"], self.ch[l], self.ch[l]) if l < top else T(B["bot"])
            self._conv(f"enc{l}b", T(B[f"t{l}"]), dst, R[l], stream=stream)
            if l < top:
                U.pu_pool(dst, T(B[f"p{l + 1}"]), stream)
        for l in reversed(range(top)):
            src = T(B["bot"]) if l == top - 1 else T(B[f"ub{l + 1}"])
            L = self.layers[f"up{l}"]
            w = self.w(L.name, self.wt)
            for q, oo in enumerate(UP8):
                U.pu_conv(src, w[q * L.cin * L.cout:], 1, ZERO1, None, T(B[f"cat{l}"], 0, self.ch[l]), R[l + 1], 1,
                          2, oo, False, False, False, stream)
            self._conv(f"dec{l}a", T(B[f"cat{l}"]), T(B[f"ua{l}"]), R[l], stream=stream)
            self._conv(f"dec{l}b", T(B[f"ua{l}"]), T(B[f"ub{l}"]), R[l], stream=stream)
        U.pu_head(T(B["ub0"]), self.w("head", self.master), self.b("head"), B["y"], stream)
        return B["y"]

    def backward(self, B, stream=None):
        """Gradients of every parameter from dL/dy in B["gy"] (after forward)."""
        T = U.tensor
        R, top = B["R"], self.levels - 1
        U.pu_head_backward(T(B["ub0"]), self.w("head", self.master), B["gy"], T(B["gub0"]),
                           self.w("head", self.grad), self.b("head", self.grad), self.small, stream)
        for l in range(top):
            U.pu_relu_backward(T(B[f"ub{l}"]), T(B[f"gub{l}"]), stream)
            self._conv_back(f"dec{l}b", T(B[f"ua{l}"]), T(B[f"gub{l}"]), T(B[f"gua{l}"]), R[l], B, stream)
            U.pu_relu_backward(T(B[f"ua{l}"]), T(B[f"gua{l}"]), stream)
            self._conv_back(f"dec{l}a", T(B[f"cat{l}"]), T(B[f"gua{l}"]), T(B[f"gcat{l}"]), R[l], B, stream)
            # transposed convolution: data gradient gathers the 8 children, weights per child parity
            src, gsrc = ("bot", "gbot") if l == top - 1 else (f"ub{l + 1}", f"gub{l + 1}")
            L = self.layers[f"up{l}"]
            gup = T(B[f"gcat{l}"], 0, self.ch[l])
            U.pu_conv(gup, self.w(L.name), 8, UP8, None, T(B[gsrc]), R[l + 1], 2, 1, (0, 0, 0), False,
                      False, False, stream)
            gw = self.w(L.name, self.grad)
            for q, oo in enumerate(UP8):
                U.pu_conv_wgrad(T(B[src]), gup, 1, ZERO1, gw[q * L.cin * L.cout:], None, R[l + 1], 1, 2, oo,
                                B["work"], stream)
        for l in reversed(range(self.levels)):
            out, gout = (T(B["bot"]), T(B["gbot"])) if l == top else \
                (T(B[f"cat{l}"], self.ch[l], self.ch[l]), T(B[f"gcat{l}"], self.ch[l], self.ch[l]))
            U.pu_relu_backward(out, gout, stream)
            self._conv_back(f"enc{l}b", T(B[f"t{l}"]), gout, T(B[f"gt{l}"]), R[l], B, stream)
            U.pu_relu_backward(T(B[f"t{l}"]), T(B[f"gt{l}"]), stream)
            src = T(B["x0"]) if l == 0 else T(B[f"p{l}"])
            self._conv_back(f"enc{l}a", src, T(B[f"gt{l}"]), None if l == 0 else T(B[f"gp{l}"]), R[l], B, stream)
            if l > 0:
                # the pooled features' gradient joins the skip connection's
                U.pu_pool_backward(T(B[f"gp{l}"]), T(B[f"gcat{l - 1}"], self.ch[l - 1], self.ch[l - 1]), True,
                                   stream)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        U.pu_adam(self.master, self.grad, self.m, self.v, self.wb, self.nparams, lr, beta1, beta2, eps,
                  self.step_count, stream)
        self._refresh_transposed()

    def train_step(self, B, target, lr, stream=None):
        self.forward(B, stream)
        U.pu_mse(B["y"], target, None, B["y"].numel(), self.loss, B["gy"], self.small, stream)
        self.backward(B, stream)
        self.adam_step(lr, stream=stream)
        return self.loss


# --------------------------------------------------------------------- driver
def _net_scale(spacing, factor):
    return float(spacing[0]) * factor


class WarmStart:
    """Guess {P^0} for a plan: a trained network at grid/factor and, with
    ``coarse``, a solve of the same problem on that coarse grid.

    Network only: the network's output, trilinearly upsampled.

    ``coarse``: the gradient field is block-averaged onto the network grid
    (grid / factor), that coarse problem is solved with the fixed-point CG
    variant (PI_FIXED_POINT_CG, to eps_R <= coarse_tol) starting from the
    network's output (or from zero when ``net`` is None), and the coarse
    answer is upsampled.  In Eq. MatrixEquation the previous iterate enters
    only through [W^n], whose weights count rays that start at the
    neighbour, i.e. at cells on the edge of the data: after the first outer
    step the iteration depends on the start only through its values there.
    The coarse solve gives those values to second order once the upsampling
    continues linearly to the grid's edge (pu_upsample_output); the network
    is a good start for the coarse CG, which treats all scales alike.
    FP32 plans without a mask only."""

    def __init__(self, net: UNet | None, factor: int, coarse: bool = False, coarse_tol: float = 1e-6):
        if net is None and not coarse:
            raise ValueError("a warm start needs a network or the coarse solve")
        self.net, self.factor = net, int(factor)
        self.coarse, self.coarse_tol = bool(coarse), float(coarse_tol)
        dev = net.device if net is not None else torch.device("cuda:0")
        self._rms = torch.zeros(1, dtype=torch.float32, device=dev)
        self._small = net.small if net is not None else torch.zeros(U.RMS_WORK_FLOATS, dtype=torch.float32, device=dev)
        self._coarse = {}  # (dims, spacing) -> (plan, gradient buffers, P buffer)
        self.last = {}     # what the last guess did (coarse outer/inner steps)

    def _coarse_for(self, plan: Plan, device):
        f = self.factor
        cdims = tuple(d // f for d in plan.dims)
        key = (cdims, plan.spacing)
        if key not in self._coarse:
            cp = Plan(cdims, tuple(h * f for h in plan.spacing), fixed_point=True)
            cp.autotune(reps=3)
            shape = cp.shape
            gc = [torch.zeros(shape, dtype=torch.float32, device=device) for _ in range(plan.ndim)]
            self._coarse[key] = (cp, gc, torch.zeros(shape, dtype=torch.float32, device=device))
        return self._coarse[key]

    def guess(self, plan: Plan, grads, P, mask=None, stream=None):
        nx, ny, nz = (tuple(plan.dims) + (1,))[:3]
        f = self.factor
        if self.net is not None and plan.ndim != 3:
            raise ValueError("the warm-start network is 3-D")
        if self.coarse and (plan.fp64 or mask is not None):
            raise ValueError("the coarse solve of the warm start takes FP32 plans without a mask")
        count = nx * ny * nz
        y = None
        if self.net is not None:
            res = (nz // f, ny // f, nx // f)
            B = self.net.buffers(1, res)
            U.pu_grad_rms(grads[0], grads[1], grads[2], mask, count, self._rms, self._small, stream)
            rms = float(self._rms.item())
            if not rms > 0.0:
                raise ValueError("gradient field is zero")
            U.pu_prepare_input(grads[0], grads[1], grads[2], mask, plan.dims, f, 1.0 / rms, U.tensor(B["x0"]),
                               stream)
            y = self.net.forward(B, stream)
            yscale = rms * _net_scale(plan.spacing, f)
        if not self.coarse:
            U.pu_upsample_output(y, plan.dims, f, yscale, P, plan.fp64, stream)
            return P
        cp, gc, Pc = self._coarse_for(plan, grads[0].device)
        U.pu_block_mean(grads[0], grads[1], grads[2] if plan.ndim == 3 else None, None, plan.dims, f, gc[0], gc[1],
                        gc[2] if plan.ndim == 3 else None, stream)
        if y is not None:  # the network's answer on the coarse grid starts the coarse solve
            U.pu_upsample_output(y, cp.dims, 1, yscale, Pc, False, stream)
        r = cp.solve(gc, P=Pc, tol=self.coarse_tol, max_iter=1000, warm_start=y is not None, stream=stream)
        self.last = {"coarse_outer": r.info["outer_iters"], "coarse_inner": r.info["inner_iters_total"],
                     "coarse_eps_R": r.info["eps_R"]}
        U.pu_upsample_output(Pc, plan.dims, f, 1.0, P, plan.fp64, stream)
        return P

    def close(self):
        for cp, _, _ in self._coarse.values():
            cp.close()
        self._coarse.clear()

    def solve(self, plan: Plan, grads, P=None, tol=1e-6, max_iter=10**7, mask=None):
        if P is None:
            P = torch.empty(plan.shape, dtype=plan.dtype, device=grads[0].device)
        self.guess(plan, grads, P, mask)
        return plan.solve(grads, P=P, tol=tol, max_iter=max_iter, warm_start=True)


# ------------------------------------------------------------------- training
def make_dataset(n, count, seed_base, tol=1e-6, chunk=32, device="cuda:0", noise=0.05, log=None,
                 fixed_point=False):
    """Method-generated training pairs on n^3 unit-cube grids of Gaussian-blob
    fields: network input (gradient / RMS, data fraction) and target (the
    solver's gauge-fixed pressure / (RMS * cell size)).  fixed_point: solve
    with the PI_FIXED_POINT_CG variant, which reaches the same fixed point of
    Eq. MatrixEquation in a fraction of the time."""
    import synth

    x = torch.zeros((count, n, n, n, 4), dtype=BF16, device=device)
    tgt = torch.zeros((count, n, n, n), dtype=torch.float32, device=device)
    stats = []
    rms = torch.zeros(1, dtype=torch.float32, device=device)
    small = torch.zeros(U.RMS_WORK_FLOATS, dtype=torch.float32, device=device)
    pool = []  # one plan (and so one workspace) per instance of a batch
    t0 = time.time()
    for c0 in range(0, count, chunk):
        ids = list(range(c0, min(count, c0 + chunk)))
        works = [synth.config_blobs_3d(n, noise=noise, seed=seed_base + i, device=device) for i in ids]
        grads = [[g.float().contiguous() for g in w.grads] for w in works]
        while len(pool) < len(ids):
            pool.append(Plan(works[0].dims, works[0].spacing, fixed_point=fixed_point))
        rc, Ps, infos = solve_batched(pool[:len(ids)], grads, tol=tol, max_iter=200000)
        for k, i in enumerate(ids):
            g = grads[k]
            U.pu_grad_rms(g[0], g[1], g[2], None, n ** 3, rms, small)
            r = float(rms.item())
            xi = x[i:i + 1]
            U.pu_prepare_input(g[0], g[1], g[2], None, works[k].dims, 1, 1.0 / r, U.tensor(xi))
            U.pu_upsample_output(Ps[k], works[k].dims, 1, 1.0 / (r * _net_scale(works[k].spacing, 1)), tgt[i])
            stats.append(infos[k])
        if log:
            log(f"dataset {ids[-1] + 1}/{count} solves ({time.time() - t0:.1f}s, "
                f"outer {infos[0]['outer_iters']}, eps_R {infos[0]['eps_R']:.2e})")
    torch.cuda.synchronize()
    for p in pool:
        p.close()
    return x, tgt, stats


_CH_OF_AXIS = (2, 1, 0)  # grid axes (z, y, x) -> gradient channel


def _symmetry(x, t, gen):
    """A random element of the cube's symmetry group applied to a batch:
    axis permutation and reflections of the grid, with the gradient
    components permuted and negated alongside (the pressure is a scalar and
    only moves).  The method is equivariant under these maps on isotropic
    cubic grids, so every training pair yields 48."""
    perm = torch.randperm(3, generator=gen).tolist()
    flips = [bool(torch.randint(0, 2, (1,), generator=gen).item()) for _ in range(3)]
    x = x.permute(0, 1 + perm[0], 1 + perm[1], 1 + perm[2], 4)
    t = t.permute(0, 1 + perm[0], 1 + perm[1], 1 + perm[2])
    idx = [0, 0, 0, 3]
    for k in range(3):
        idx[_CH_OF_AXIS[k]] = _CH_OF_AXIS[perm[k]]
    x = x[..., idx]
    dims = [1 + k for k in range(3) if flips[k]]
    if dims:
        x, t = x.flip(dims), t.flip(dims)
        sign = torch.ones(4, dtype=x.dtype, device=x.device)
        for k in range(3):
            if flips[k]:
                sign[_CH_OF_AXIS[k]] = -1
        x = x * sign
    return x, t


def train(net: UNet, x, tgt, steps, batch=4, lr=1e-3, seed=0, log=None, log_every=100, augment=True):
    """Adam on the mean squared error; cosine learning-rate decay; random
    cube symmetries of the training pairs (cubic grids)."""
    count = x.shape[0]
    res = tuple(x.shape[1:4])
    B = net.buffers(batch, res)
    g = torch.Generator().manual_seed(seed)
    t0 = time.time()
    hist = []
    target = torch.empty((batch,) + res, dtype=torch.float32, device=x.device)
    cubic = res[0] == res[1] == res[2]
    for s in range(steps):
        idx = torch.randint(0, count, (batch,), generator=g).to(x.device)
        xb, tb = x.index_select(0, idx), tgt.index_select(0, idx)
        if augment and cubic:
            xb, tb = _symmetry(xb, tb, g)
        B["x0"].copy_(xb)
        target.copy_(tb)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps)))
        net.train_step(B, target, lr_s)
        if log and (s % log_every == 0 or s == steps - 1):
            loss = float(net.loss.item())
            hist.append((s, loss))
            log(f"train step {s}/{steps} loss {loss:.4e} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return hist
