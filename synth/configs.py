"""The workloads the solver is exercised on, as seeded recipes.

Each recipe returns a :class:`Workload`: grid sizes, spacing, a uint8 mask
(1 = data present) and the gradient components, with NaN written into masked
cells as the paper encodes missing vectors.  The recipes stand in for the
paper's data sets (Taylor vortex, JHU isotropic turbulence cut-outs, planar
and scanning PIV), which are not available here.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import fields as F


@dataclass
class Workload:
    name: str
    dims: tuple            # (nx, ny[, nz])
    spacing: tuple         # (dx, dy[, dz])
    mask: Optional[torch.Tensor]   # uint8, storage order, 1 = valid; None = all valid
    grads: List[torch.Tensor]      # storage order, NaN in masked cells
    P_true: Optional[torch.Tensor] = None
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.dims)

    @property
    def ncells(self):
        n = 1
        for d in self.dims:
            n *= int(d)
        return n

    def to(self, device, dtype=None):
        g = [x.to(device=device, dtype=dtype or x.dtype) for x in self.grads]
        m = None if self.mask is None else self.mask.to(device)
        P = None if self.P_true is None else self.P_true.to(device=device, dtype=dtype or self.P_true.dtype)
        return Workload(self.name, self.dims, self.spacing, m, g, P, dict(self.meta))


def _apply_mask(grads, mask):
    if mask is None:
        return grads
    bad = mask == 0
    out = []
    for g in grads:
        g = g.clone()
        g[bad] = float("nan")
        out.append(g)
    return out


def config_sin64(n=64, noise=0.05, seed=1, device="cpu"):
    """P = sin(2 pi x) cos(2 pi y) on [0,1]^2 sampled at n^2 centres, unit
    spacing: the solver sees spacing 1 and the per-cell gradient h * grad P
    (h = 1/n), which is the same problem as spacing h with grad P."""
    P, g, (h, _) = F.sin_cos_2d((n, n), device=device)
    g = [h * x for x in g]
    g = F.add_noise(g, None, noise, seed, device=device)
    return Workload("sin64", (n, n), (1.0, 1.0), None, g, P, dict(seed=seed, noise=noise))


def config_lamb_oseen_2d(n=2048, noise=0.10, seed=2, mask_frac=0.05, device="cpu",
                         with_pressure=False):
    """Lamb-Oseen pair (core radius 0.05, circulations +1/-1, centres
    U[0.2,0.8]^2), 10 % gradient noise, random disks covering >= 5 % of the
    cells (radii U[0.01, 0.04])."""
    P, g, spacing = F.lamb_oseen_pair((n, n), seed, rc=0.05, device=device,
                                      with_pressure=with_pressure and str(device) == "cpu")
    mask = F.disk_mask((n, n), seed, frac=mask_frac, device=device) if mask_frac > 0 else None
    g = F.add_noise(g, mask, noise, seed, device=device)
    return Workload("lamb_oseen_2d", (n, n), spacing, mask, _apply_mask(g, mask), P,
                    dict(seed=seed, noise=noise, mask_frac=mask_frac))


def config_blobs_3d(n=500, noise=0.05, seed=3, device="cpu", with_pressure=False, nblobs=32,
                    mask_frac=0.0):
    """Sum of 32 Gaussian pressure blobs (centres U[0,1]^3, widths
    U[0.02, 0.1], amplitudes N(0,1)) on an n^3 grid, 5 % gradient noise."""
    dims = (n, n, n) if np.isscalar(n) else tuple(n)
    P, g, spacing = F.gaussian_blobs(dims, seed, nblobs=nblobs, device=device,
                                     with_pressure=with_pressure)
    mask = F.disk_mask(dims, seed, frac=mask_frac, rmin=0.03, rmax=0.1, device=device) if mask_frac > 0 else None
    g = F.add_noise(g, mask, noise, seed, device=device)
    return Workload("blobs_3d", dims, spacing, mask, _apply_mask(g, mask), P,
                    dict(seed=seed, noise=noise))


def batched_instances(count2d=512, count3d=16, seed_base=4000, side2d=(128, 1024),
                      side3d=(64, 256), noise=0.05, device="cpu"):
    """Uneven batch: 2-D snapshots with sides iid U{side2d}, 2-8 Lamb-Oseen
    vortices (Gamma = +-U[0.5,1.5], rc ~ U[0.02,0.08]) and a 0-5 % disk mask,
    plus 3-D volumes with sides iid U{side3d} and 32 Gaussian blobs.  Instance
    i uses seed seed_base + i."""
    out = []
    for i in range(count2d + count3d):
        seed = seed_base + i
        rng = np.random.default_rng(seed)
        if i < count2d:
            nx, ny = (int(v) for v in rng.integers(side2d[0], side2d[1] + 1, size=2))
            k = int(rng.integers(2, 9))
            centers = rng.uniform(0.1, 0.9, size=(k, 2))
            gam = rng.uniform(0.5, 1.5, size=k) * rng.choice([-1.0, 1.0], size=k)
            rcs = rng.uniform(0.02, 0.08, size=k)
            _, g, spacing = F.lamb_oseen_vortices((nx, ny), centers, gam, rcs, device=device)
            frac = float(rng.uniform(0.0, 0.05))
            mask = F.disk_mask((nx, ny), seed, frac=frac, device=device) if frac > 0.005 else None
            g = F.add_noise(g, mask, noise, seed, device=device)
            out.append(Workload(f"b2d_{i}", (nx, ny), spacing, mask, _apply_mask(g, mask), None,
                                dict(seed=seed)))
        else:
            dims = tuple(int(v) for v in rng.integers(side3d[0], side3d[1] + 1, size=3))
            _, g, spacing = F.gaussian_blobs(dims, seed, device=device, with_pressure=False)
            g = F.add_noise(g, None, noise, seed, device=device)
            out.append(Workload(f"b3d_{i}", dims, spacing, None, g, None, dict(seed=seed)))
    return out


def random_small(seed, ndim, dims: Sequence[int], anisotropic=True, mask_frac=0.1,
                 noise=0.05, device="cpu"):
    """Small parity case: Gaussian blobs on a grid with random spacing and a
    random disk mask."""
    rng = np.random.default_rng(seed)
    if anisotropic:
        lengths = tuple(float(v) for v in rng.uniform(0.5, 2.0, size=ndim))
    else:
        lengths = (1.0,) * ndim
    P, g, _ = F.gaussian_blobs(tuple(dims), seed, nblobs=8, sigma_range=(0.08, 0.3), device=device)
    spacing = tuple(lengths[a] / dims[a] for a in range(ndim))
    # stretch the unit-domain field onto the physical lengths: d/dx_phys = d/dx / L
    g = [g[a] / lengths[a] for a in range(ndim)]
    mask = F.disk_mask(tuple(dims), seed, frac=mask_frac, rmin=0.05, rmax=0.15,
                       device=device) if mask_frac > 0 else None
    g = F.add_noise(g, mask, noise, seed, device=device)
    return Workload(f"small{ndim}d_{seed}", tuple(dims), spacing, mask, _apply_mask(g, mask), P,
                    dict(seed=seed))
