"""Analytic pressure fields with exact gradients, seeded noise and masks.

Arrays follow the library's storage order: a grid with sizes (nx, ny[, nz])
is held as an array of shape (ny, nx) or (nz, ny, nx), so x is the fastest
index.  Cells are centred: the i-th centre along an axis of length Lx with nx
cells sits at (i + 1/2) * Lx / nx.

Generators run in torch on any device, so the 125 M-cell volumes can be built
directly in GPU memory; the small parameter draws (centres, radii,
amplitudes) always come from a seeded numpy generator so that the same seed
gives the same field on every device.  Gradient noise is drawn from a seeded
torch generator on the target device.
"""

from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import torch


def _axes(shape: Sequence[int], lengths: Sequence[float] | None, origin, device, dtype):
    """Per-axis 1-D centre coordinates, reshaped to broadcast against the
    storage-order array (axis 0 of the array is the slowest grid axis)."""
    nd = len(shape)
    if lengths is None:
        lengths = [1.0] * nd
    if origin is None:
        origin = [0.0] * nd
    out = []
    for a in range(nd):
        n = int(shape[a])
        h = float(lengths[a]) / n
        c = (torch.arange(n, device=device, dtype=dtype) + 0.5) * h + float(origin[a])
        view = [1] * nd
        view[nd - 1 - a] = n  # x is the last array axis
        out.append(c.view(view))
    return out


def cell_centers(shape, lengths=None, origin=None, device="cpu", dtype=torch.float64):
    """Broadcastable cell-centre coordinates (x, y[, z]) and the spacings."""
    nd = len(shape)
    if lengths is None:
        lengths = [1.0] * nd
    spacing = tuple(float(lengths[a]) / int(shape[a]) for a in range(nd))
    return _axes(shape, lengths, origin, device, dtype), spacing


def _full(t, shape_np):
    return t.expand(*shape_np).contiguous()


def sin_cos_2d(shape, device="cpu", dtype=torch.float64):
    """P = sin(2 pi x) cos(2 pi y) on the unit square."""
    (x, y), spacing = cell_centers(shape, device=device, dtype=dtype)
    tp = 2.0 * math.pi
    P = torch.sin(tp * x) * torch.cos(tp * y)
    gx = tp * torch.cos(tp * x) * torch.cos(tp * y)
    gy = -tp * torch.sin(tp * x) * torch.sin(tp * y)
    s = (shape[1], shape[0])
    return _full(P, s), [_full(gx, s), _full(gy, s)], spacing


def quadratic(shape, seed, spacing=None, device="cpu", dtype=torch.float64):
    """A random polynomial of total degree two, P = c + g.x + x.H.x / 2.

    The trapezoid face rule is exact for such fields, so their gradients are
    integrable without discretisation error."""
    nd = len(shape)
    rng = np.random.default_rng(seed)
    c0 = rng.normal()
    g = rng.normal(size=nd)
    H = rng.normal(size=(nd, nd))
    H = 0.5 * (H + H.T)
    if spacing is None:
        spacing = [1.0 / n for n in shape]
    lengths = [spacing[a] * shape[a] for a in range(nd)]
    X, _ = cell_centers(shape, lengths=lengths, device=device, dtype=dtype)
    P = torch.zeros((), device=device, dtype=dtype) + c0
    grads = []
    for a in range(nd):
        P = P + g[a] * X[a]
        for b in range(nd):
            P = P + 0.5 * H[a, b] * X[a] * X[b]
    for a in range(nd):
        ga = torch.zeros((), device=device, dtype=dtype) + g[a]
        for b in range(nd):
            ga = ga + H[a, b] * X[b]
        grads.append(ga)
    s = tuple(reversed([int(n) for n in shape]))
    return _full(P, s), [_full(q, s) for q in grads], tuple(spacing)


def _lamb_oseen_pressure_np(r2, gamma, rc, rho=1.0):
    from scipy.special import exp1

    xi = np.maximum(r2 / rc**2, 1e-300)
    core = -np.expm1(-xi)
    return -rho * gamma**2 / (8 * math.pi**2 * rc**2) * (core**2 / xi + 2 * exp1(xi) - 2 * exp1(2 * xi))


def lamb_oseen_vortices(shape, centers, gammas, rcs, device="cpu", dtype=torch.float64,
                        with_pressure=False, rho=1.0):
    """Superposed Lamb-Oseen pressure wells on the unit square.

    Each vortex contributes P_k(r) with dP_k/dr = rho u_theta^2 / r,
    u_theta = Gamma / (2 pi r) (1 - exp(-r^2 / rc^2)), so the gradient field is
    the exact gradient of the summed pressure (the sign of Gamma drops out).
    The pressure itself (needed only for accuracy checks) uses scipy's E1 and
    is only built on the CPU."""
    (x, y), spacing = cell_centers(shape, device=device, dtype=dtype)
    s = (shape[1], shape[0])
    gx = torch.zeros(s, device=device, dtype=dtype)
    gy = torch.zeros(s, device=device, dtype=dtype)
    P = np.zeros(s) if with_pressure else None
    for (cx, cy), gam, rc in zip(centers, gammas, rcs):
        dx = x - cx
        dy = y - cy
        r2 = dx * dx + dy * dy
        xi = r2 / rc**2
        # rho u^2 / r^2 times the displacement gives the radial gradient.
        one_m = -torch.expm1(-xi)
        # u_theta^2 / r^2 = Gamma^2 (1-e^-xi)^2 / (4 pi^2 r^4); for r -> 0 use the
        # series (1-e^-xi)/r^2 -> 1/rc^2.
        safe = torch.where(r2 > 0, r2, torch.ones_like(r2))
        ratio = torch.where(r2 > 1e-30 * rc**2, one_m / safe, torch.full_like(r2, 1.0 / rc**2))
        fac = rho * gam**2 / (4 * math.pi**2) * ratio * ratio
        gx = gx + fac * dx
        gy = gy + fac * dy
        if with_pressure:
            xn = x.cpu().numpy() - cx
            yn = y.cpu().numpy() - cy
            P = P + _lamb_oseen_pressure_np(xn**2 + yn**2, gam, rc, rho)
    Pt = torch.as_tensor(P, dtype=dtype) if with_pressure else None
    return Pt, [gx, gy], spacing


def lamb_oseen_pair(shape, seed, rc=0.05, device="cpu", dtype=torch.float64, with_pressure=False):
    """Two Lamb-Oseen vortices, circulations +1 and -1, centres U[0.2, 0.8]^2."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.2, 0.8, size=(2, 2))
    return lamb_oseen_vortices(shape, centers, [1.0, -1.0], [rc, rc], device=device, dtype=dtype,
                               with_pressure=with_pressure)


def gaussian_blobs(shape, seed, nblobs=32, sigma_range=(0.02, 0.1), device="cpu",
                   dtype=torch.float64, with_pressure=True, t=0.0, speed=0.0):
    """P = sum_k a_k exp(-|x - c_k|^2 / (2 sigma_k^2)) on the unit square/cube,
    c_k ~ U[0,1]^d, sigma_k ~ U[sigma_range], a_k ~ N(0, 1).  With speed > 0
    the blobs drift: c_k(t) = c_k + t v_k, v_k ~ N(0, speed^2) per axis (drawn
    after the other parameters, so t = 0 gives the static field of the seed)."""
    nd = len(shape)
    rng = np.random.default_rng(seed)
    cs = rng.uniform(0.0, 1.0, size=(nblobs, nd))
    sig = rng.uniform(sigma_range[0], sigma_range[1], size=nblobs)
    amp = rng.normal(size=nblobs)
    if speed > 0.0:
        cs = cs + t * rng.normal(0.0, speed, size=(nblobs, nd))
    X, spacing = cell_centers(shape, device=device, dtype=dtype)
    s = tuple(reversed([int(n) for n in shape]))
    P = torch.zeros(s, device=device, dtype=dtype) if with_pressure else None
    grads = [torch.zeros(s, device=device, dtype=dtype) for _ in range(nd)]
    for k in range(nblobs):
        # separable exponentials keep the 125 M-cell build cheap
        facs = [torch.exp(-((X[a] - cs[k, a]) ** 2) / (2 * sig[k] ** 2)) for a in range(nd)]
        e = facs[0]
        for a in range(1, nd):
            e = e * facs[a]
        if with_pressure:
            P.add_(amp[k] * e)
        for a in range(nd):
            grads[a].add_(e * (-(X[a] - cs[k, a]) * (amp[k] / sig[k] ** 2)))
    return P, grads, spacing


def taylor_vortex(shape, t=0.1, half_width=3.0, device="cpu", dtype=torch.float64):
    """Decaying Taylor vortex in the paper's normalised units (H = nu = rho = 1),
    on the square [-half_width, half_width]^2 (Section 'Taylor Vortex (2D)'):
    P(r) = -exp(-r^2 / (2 t)) / (64 pi^2 t^3)."""
    L = 2 * half_width
    X, spacing = cell_centers(shape, lengths=[L, L], origin=[-half_width, -half_width],
                              device=device, dtype=dtype)
    x, y = X
    r2 = x * x + y * y
    amp = 1.0 / (64 * math.pi**2 * t**3)
    P = -amp * torch.exp(-r2 / (2 * t))
    dPdr_over_r = amp / t * torch.exp(-r2 / (2 * t))
    s = (shape[1], shape[0])
    return _full(P, s), [_full(dPdr_over_r * x, s), _full(dPdr_over_r * y, s)], spacing


def add_noise(grads, mask, pct, seed, device=None):
    """Add iid Gaussian noise to every gradient component, with standard
    deviation pct * RMS(|grad|) taken over the valid cells."""
    if pct == 0:
        return [g.clone() for g in grads]
    device = grads[0].device if device is None else device
    valid = None if mask is None else (mask != 0)
    mag2 = torch.zeros_like(grads[0])
    for g in grads:
        mag2 = mag2 + g * g
    if valid is not None:
        rms = torch.sqrt(mag2[valid].mean())
    else:
        rms = torch.sqrt(mag2.mean())
    sigma = float(pct) * float(rms)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = []
    for g in grads:
        n = torch.randn(g.shape, generator=gen, device=device, dtype=g.dtype)
        out.append(g + sigma * n)
    return out


def disk_mask(shape, seed, frac=0.05, rmin=0.01, rmax=0.04, device="cpu"):
    """Union of random disks (balls in 3D) on the unit domain, added until at
    least ``frac`` of the cells are masked.  Returns uint8, 1 = valid."""
    nd = len(shape)
    rng = np.random.default_rng(seed)
    X, _ = cell_centers(shape, device=device, dtype=torch.float32)
    s = tuple(reversed([int(n) for n in shape]))
    masked = torch.zeros(s, dtype=torch.bool, device=device)
    total = masked.numel()
    count = 0
    while count < frac * total:
        c = rng.uniform(0.0, 1.0, size=nd)
        r = rng.uniform(rmin, rmax)
        d2 = None
        for a in range(nd):
            t = (X[a] - float(c[a])) ** 2
            d2 = t if d2 is None else d2 + t
        masked |= (d2 <= r * r).expand(s)
        count = int(masked.sum())
    return (~masked).to(torch.uint8)
