"""FP64 reference of the velocity -> pressure-gradient stage (the source field
f that the integration consumes), written out from the paper's equations.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays are in storage
order ([z, y, x] in 3-D, [y, x] in 2-D); component k of a vector field is the
derivative / velocity along axis x, y, z for k = 0, 1, 2; spacing = (dx, dy[, dz]).

* ns_source: incompressible Navier-Stokes, Eq. (1) of the introduction:
  grad P = -rho (du/dt + (u . grad) u) + mu lap u.
* rans_source: Reynolds-averaged momentum without viscous terms (Eq. RANS_f):
  f_i = -rho (U_j dU_i/dx_j + d(R_ij)/dx_j).
* compressible_source: the compressible RANS form of the supersonic
  double-fin section (Eq. compressible-pressure), solved for
  grad ln(P / P_inf): (delta_ij + W_ij / (R T)) g_j = -(1/(R T)) (dW_ij/dx_j
  - W_ij / T dT/dx_j) with W_ij = U_i U_j + R_ij and the adiabatic temperature
  T / T_inf = 1 + (gamma - 1)/2 M_inf^2 (1 - V^2 / V_inf^2).

Derivatives are second-order central differences, with second-order
one-sided differences at the grid ends (the paper computes its source terms
with second-order central differences); second derivatives use the
three-point rule inside and a four-point one-sided rule at the ends.
"""

from __future__ import annotations

import numpy as np


def _axis(ndim, k):
    """numpy axis of physical axis k (0 = x) for storage-order arrays."""
    return ndim - 1 - k


def d1(f, h, k):
    """df/dx_k: (f[i+1] - f[i-1]) / 2h inside, (-3 f0 + 4 f1 - f2) / 2h and
    its mirror at the ends; first order for 2 cells, 0 for 1."""
    f = np.asarray(f, float)
    ax = _axis(f.ndim, k)
    n = f.shape[ax]
    out = np.zeros_like(f)
    if n == 1:
        return out
    g = np.moveaxis(f, ax, 0)
    o = np.moveaxis(out, ax, 0)
    if n == 2:
        o[0] = o[1] = (g[1] - g[0]) / h
        return out
    o[1:-1] = (g[2:] - g[:-2]) / (2 * h)
    o[0] = (-3 * g[0] + 4 * g[1] - g[2]) / (2 * h)
    o[-1] = (3 * g[-1] - 4 * g[-2] + g[-3]) / (2 * h)
    return out


def d2(f, h, k):
    """d2f/dx_k^2: (f[i+1] - 2 f[i] + f[i-1]) / h^2 inside, (2 f0 - 5 f1 + 4 f2
    - f3) / h^2 and its mirror at the ends (4 cells or more); 3 cells: the
    interior value at the ends too; fewer: 0."""
    f = np.asarray(f, float)
    ax = _axis(f.ndim, k)
    n = f.shape[ax]
    out = np.zeros_like(f)
    if n < 3:
        return out
    g = np.moveaxis(f, ax, 0)
    o = np.moveaxis(out, ax, 0)
    o[1:-1] = (g[2:] - 2 * g[1:-1] + g[:-2]) / h ** 2
    if n == 3:
        o[0] = o[2] = o[1]
    else:
        o[0] = (2 * g[0] - 5 * g[1] + 4 * g[2] - g[3]) / h ** 2
        o[-1] = (2 * g[-1] - 5 * g[-2] + 4 * g[-3] - g[-4]) / h ** 2
    return out


def ns_source(u, spacing, rho, mu, dudt=None):
    """-rho (du/dt + (u . grad) u) + mu lap u, u a list of ndim components."""
    nd = len(u)
    f = []
    for i in range(nd):
        conv = sum(u[j] * d1(u[i], spacing[j], j) for j in range(nd))
        lap = sum(d2(u[i], spacing[j], j) for j in range(nd))
        dt = 0.0 if dudt is None else dudt[i]
        f.append(-rho * (dt + conv) + mu * lap)
    return f


def time_derivative(u_prev, u_next, dt):
    """Central difference of two snapshots 2 dt apart."""
    return [(b - a) / (2 * dt) for a, b in zip(u_prev, u_next)]


def stress_index(i, j, nd):
    """Position of R_ij in the list of independent Reynolds stresses:
    2-D (uu, vv, uv), 3-D (uu, vv, ww, uv, uw, vw)."""
    if i == j:
        return i
    a, b = min(i, j), max(i, j)
    if nd == 2:
        return 2
    return {(0, 1): 3, (0, 2): 4, (1, 2): 5}[(a, b)]


def rans_source(U, spacing, rho, R=None):
    nd = len(U)
    f = []
    for i in range(nd):
        acc = sum(U[j] * d1(U[i], spacing[j], j) for j in range(nd))
        if R is not None:
            acc = acc + sum(d1(R[stress_index(i, j, nd)], spacing[j], j) for j in range(nd))
        f.append(-rho * acc)
    return f


def temperature(U, gamma, T_inf, M_inf, V_inf):
    V2 = sum(c * c for c in U)
    return T_inf * (1 + 0.5 * (gamma - 1) * M_inf ** 2 * (1 - V2 / V_inf ** 2))


def compressible_source(U, spacing, gas_R, gamma, T_inf, M_inf, V_inf, R=None):
    """grad ln(P / P_inf) from the mean velocity (and Reynolds stresses), by a
    per-cell linear solve (numpy.linalg.solve)."""
    nd = len(U)
    T = temperature(U, gamma, T_inf, M_inf, V_inf)
    Wij = [[U[i] * U[j] + (0.0 if R is None else R[stress_index(i, j, nd)]) for j in range(nd)]
           for i in range(nd)]
    dT = [d1(T, spacing[j], j) for j in range(nd)]
    rhs = []
    for i in range(nd):
        div = sum(d1(Wij[i][j], spacing[j], j) for j in range(nd))
        corr = sum(Wij[i][j] / T * dT[j] for j in range(nd))
        rhs.append(-(div - corr) / (gas_R * T))
    shape = U[0].shape
    A = np.zeros(shape + (nd, nd))
    for i in range(nd):
        for j in range(nd):
            A[..., i, j] = (1.0 if i == j else 0.0) + Wij[i][j] / (gas_R * T)
    b = np.stack(rhs, axis=-1)
    g = np.linalg.solve(A, b[..., None])[..., 0]
    return [g[..., i] for i in range(nd)]


def taylor_vortex(shape, spacing, t, H=1.0, nu=1.0, rho=1.0, origin=None):
    """Decaying Taylor vortex of the 2-D benchmark section: velocity,
    analytic pressure and its exact gradient on a cell-centred grid centred
    on the vortex (the caller picks spacing in units of sqrt(H))."""
    ny, nx = shape
    x = (np.arange(nx) - (nx - 1) / 2) * spacing[0]
    y = (np.arange(ny) - (ny - 1) / 2) * spacing[1]
    X, Y = np.meshgrid(x, y)
    r2 = X * X + Y * Y
    ut_over_r = H / (8 * np.pi * nu * t * t) * np.exp(-r2 / (4 * nu * t))
    u, v = -Y * ut_over_r, X * ut_over_r
    P = -rho * H * H / (64 * np.pi ** 2 * nu * t ** 3) * np.exp(-r2 / (2 * nu * t))
    dPdr_over_r = rho * H * H / (64 * np.pi ** 2 * nu * t ** 3) * np.exp(-r2 / (2 * nu * t)) / (nu * t)
    return [u, v], P, [X * dPdr_over_r, Y * dPdr_over_r]


def taylor_vortex_dudt(shape, spacing, t, H=1.0, nu=1.0):
    """Exact time derivative of the Taylor-vortex velocity."""
    ny, nx = shape
    x = (np.arange(nx) - (nx - 1) / 2) * spacing[0]
    y = (np.arange(ny) - (ny - 1) / 2) * spacing[1]
    X, Y = np.meshgrid(x, y)
    r2 = X * X + Y * Y
    a = H / (8 * np.pi * nu)
    # d/dt [t^-2 exp(-r2 / (4 nu t))] = exp(...) (-2 t^-3 + r2 / (4 nu) t^-4)
    g = a * np.exp(-r2 / (4 * nu * t)) * (-2.0 / t ** 3 + r2 / (4 * nu * t ** 4))
    return [-Y * g, X * g]
