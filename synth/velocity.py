"""Analytic velocity fields and the velocity-noise models of the paper.

Inputs of the velocity -> source stage.  Like the rest of this package it
holds none of the integration method's arithmetic: fields, their exact
pressures, and seeded noise.  Arrays are in storage order (x fastest); cells
are centred as in ``synth.fields``.

* taylor_velocity: the decaying Taylor vortex of Section "Taylor Vortex
  (2D)" in normalised units (H = nu = rho = 1).
* abc_velocity: the Arnold-Beltrami-Childress flow on a 2 pi periodic box,
  decaying as exp(-nu t).  It is a Beltrami field with curl u = u, so
  lap u = -u and (u . grad) u = grad(|u|^2 / 2): with mu = rho nu it solves
  the incompressible Navier-Stokes equations exactly, with pressure
  P = -rho |u|^2 / 2 (up to a constant).  It serves as the 3-D analogue of
  the Taylor vortex.
* noise_angular: Eq. NoisyVectorsTheta, u + s n |u| with n a unit vector of
  uniformly distributed direction.
* noise_multiplicative: Eq. NoisyVectors, u (1 + s n); n is one standard
  normal number per cell, so a vector is rescaled and keeps its direction.
"""

from __future__ import annotations

import math
from typing import Sequence

import torch

from .fields import cell_centers


def _full(t, shape_np):
    return t.expand(*shape_np).contiguous()


def taylor_velocity(shape, t=1.0, half_width=3.0, device="cpu", dtype=torch.float64):
    """(u, v), P and spacing of the Taylor vortex centred on the square
    [-half_width, half_width]^2, sampled at cell centres."""
    L = 2 * half_width
    (x, y), spacing = cell_centers(shape, lengths=[L, L], origin=[-half_width, -half_width],
                                   device=device, dtype=dtype)
    r2 = x * x + y * y
    s = (int(shape[1]), int(shape[0]))
    ut_over_r = torch.exp(-r2 / (4 * t)) / (8 * math.pi * t * t)
    P = -torch.exp(-r2 / (2 * t)) / (64 * math.pi ** 2 * t ** 3)
    return [_full(-y * ut_over_r, s), _full(x * ut_over_r, s)], _full(P, s), spacing


def abc_velocity(shape, t=0.0, nu=1.0, rho=1.0, coeffs=(1.0, math.sqrt(2.0 / 3.0), math.sqrt(1.0 / 3.0)),
                 device="cpu", dtype=torch.float64):
    """(u, v, w), P = -rho |u|^2 / 2 and spacing of the decaying ABC flow
    u = e^{-nu t} (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)
    on [0, 2 pi]^3."""
    A, B, C = coeffs
    L = 2 * math.pi
    (x, y, z), spacing = cell_centers(shape, lengths=[L, L, L], device=device, dtype=dtype)
    d = math.exp(-nu * t)
    s = tuple(int(n) for n in reversed(shape))
    u = [_full(d * (A * torch.sin(z) + C * torch.cos(y)), s),
         _full(d * (B * torch.sin(x) + A * torch.cos(z)), s),
         _full(d * (C * torch.sin(y) + B * torch.cos(x)), s)]
    P = -0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
    return u, P, spacing


def _magnitude(u: Sequence[torch.Tensor]):
    m = torch.zeros_like(u[0])
    for c in u:
        m = m + c * c
    return torch.sqrt(m)


def noise_angular(u, s, seed):
    """u + s n |u| with n a random unit vector: a uniform angle in 2-D, a
    uniform direction on the sphere in 3-D (normalised Gaussian triple)."""
    gen = torch.Generator(device=u[0].device)
    gen.manual_seed(int(seed))
    mag = _magnitude(u)
    if len(u) == 2:
        th = 2 * math.pi * torch.rand(u[0].shape, generator=gen, device=u[0].device, dtype=u[0].dtype)
        n = [torch.cos(th), torch.sin(th)]
    else:
        g = [torch.randn(u[0].shape, generator=gen, device=u[0].device, dtype=u[0].dtype) for _ in u]
        r = _magnitude(g)
        n = [c / r for c in g]
    return [c + s * nc * mag for c, nc in zip(u, n)]


def noise_multiplicative(u, s, seed):
    """u (1 + s n), n ~ N(0, 1) drawn once per cell."""
    gen = torch.Generator(device=u[0].device)
    gen.manual_seed(int(seed))
    n = torch.randn(u[0].shape, generator=gen, device=u[0].device, dtype=u[0].dtype)
    return [c * (1 + s * n) for c in u]
