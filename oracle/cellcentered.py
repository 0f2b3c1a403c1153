"""The cell-centred scheme in 2-D: per-cell ray counters by tracing the
nearest-centre paths, and the sparse system built from them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Path (Section "Method Concept", the cell-centred scheme): a ray less steep
than the cell diagonal visits every column once and takes, in each column,
the cell whose centre is nearest to it (y rounded); a steeper ray visits
every row once with x rounded.  Consecutive cells of a path are face or
diagonal neighbours, and the pressure is carried from centre to centre with
the trapezoid rule along the segment between them,
    P_C = P_J - Delta_J . (f(J) + f(C)) / 2,
Delta_J the displacement from C to J (Eq. ExplicitEqn_FaceCrossing with the
diagonal directions of the cell-centred scheme).

Counters (the limit of infinite rays of Section "Method Concept"): A_J^i is
the measure, over all angles theta and perpendicular offsets s, of the rays
whose path reaches C with J as the previous cell.  Boundary rule, read as
for the face-crossing scheme (the ray "begins" where the data does): if the
cell before J on the path holds no data or lies outside the grid the ray
starts at J and carries J's pressure of the previous sweep (i = n), else the
current one (i = n + 1); if J itself holds no data the ray starts at C
(A_C^n).  The paper gives its cell-centred boundary weights only in
supplementary material that is not available; this is a derivation of our
own from the definition above.

Computation.  There are 8 sectors: travel along +-x or +-y (the major axis)
with the lateral coordinate rising or falling (slope sign mu).  In a sector
the angle phi from the major axis runs over (0, phi_d), tan phi_d =
h_minor / h_major.  The rays through C at angle phi have lateral offsets eta
in [-1/2, 1/2) (units of h_minor, measured where the ray crosses C's
column or row), each with measure h_minor cos(phi) d(eta) d(phi).  One step
back along the path the lateral position is eta - mu tau, two steps back
eta - 2 mu tau, tau = h_major tan(phi) / h_minor, and the previous cells are
the rounded positions.  The eta window is cut at every position where one of
the two roundings changes, so J and the cell before it are fixed on each
piece; the angle integral is a Gauss-Legendre rule on each interval between
the angles at which the set of cuts changes (where the piece lengths,
linear in tau, change form).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .system import System

# the 8 neighbours of the cell-centred scheme, (name, dx, dy)
CC_DIRECTIONS = (("E", 1, 0), ("W", -1, 0), ("N", 0, 1), ("S", 0, -1),
                 ("NE", 1, 1), ("NW", -1, 1), ("SE", 1, -1), ("SW", -1, -1))
_NAME = {(dx, dy): n for n, dx, dy in CC_DIRECTIONS}


def _valid_at(mask, dx, dy):
    """Data flag of cell (x + dx, y + dy) for every cell (y, x); outside = 0."""
    ny, nx = mask.shape
    pad = 3
    p = np.pad(mask != 0, pad, constant_values=False).astype(np.float64)
    return p[pad + dy: pad + dy + ny, pad + dx: pad + dx + nx]


def _sector_pieces(h_major, h_minor, mu, n_gl=24):
    """Yield (measure, (j_major, j_minor), (k_major, k_minor)) for one sector
    travelling along +major: offsets of J and of the cell before it relative
    to C in (major, minor) steps, and the measure of the rays of that piece
    at one quadrature node.  Also yields the window measure with key None."""
    phi_d = math.atan2(h_minor, h_major)
    # angles where a cut eta = k + 1/2 + m mu tau crosses the window ends:
    # tau = j / m for m = 1, 2
    taus = sorted({j / m for m in (1, 2) for j in range(1, 2 * m) if 0.0 < j / m < 1.0})
    phis = [0.0] + [math.atan(t * h_minor / h_major) for t in taus] + [phi_d]
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    for a, b in zip(phis[:-1], phis[1:]):
        for x, w in zip(xg, wg):
            phi = 0.5 * (a + b) + 0.5 * (b - a) * x
            wq = 0.5 * (b - a) * w * h_minor * math.cos(phi)
            tau = h_major * math.tan(phi) / h_minor
            cuts = sorted(e for m in (1, 2) for k in range(-4, 5)
                          for e in (k + 0.5 + m * mu * tau,) if -0.5 < e < 0.5)
            edges = [-0.5] + cuts + [0.5]
            yield wq, None, None
            for e0, e1 in zip(edges[:-1], edges[1:]):
                if e1 <= e0:
                    continue
                eta = 0.5 * (e0 + e1)
                r1 = math.floor(eta - mu * tau + 0.5)
                r2 = math.floor(eta - 2 * mu * tau + 0.5)
                yield wq * (e1 - e0), (-1, r1), (-2, r2)


def cc_counters(mask, spacing, n_gl=24):
    """Counters of every cell (storage-order arrays, zero at masked cells):
    {(name, 'np1'), (name, 'n')} for the 8 neighbours, 'C_n', and the scalar
    'Atot' (the measure of all rays through a cell)."""
    mask = np.asarray(mask)
    if mask.ndim != 2:
        raise ValueError("the cell-centred scheme is 2-D only")
    dx, dy = (float(s) for s in spacing)
    out = {(n, i): np.zeros(mask.shape) for n, _, _ in CC_DIRECTIONS for i in ("np1", "n")}
    out["C_n"] = np.zeros(mask.shape)
    atot = 0.0
    cache = {}

    def valid(ox, oy):
        if (ox, oy) not in cache:
            cache[(ox, oy)] = _valid_at(mask, ox, oy)
        return cache[(ox, oy)]

    for major in (0, 1):
        h_major, h_minor = (dx, dy) if major == 0 else (dy, dx)
        for sgn in (1, -1):
            for mu in (1, -1):
                for m, J, K in _sector_pieces(h_major, h_minor, mu, n_gl):
                    if J is None:
                        atot += m
                        continue
                    # (major, minor) steps -> grid (x, y) offsets; travel sign sgn
                    def xy(off):
                        maj, mnr = sgn * off[0], off[1]
                        return (maj, mnr) if major == 0 else (mnr, maj)
                    jx, jy = xy(J)
                    kx, ky = xy(K)
                    vj, vk = valid(jx, jy), valid(kx, ky)
                    name = _NAME[(jx, jy)]
                    out[(name, "np1")] += m * vj * vk
                    out[(name, "n")] += m * vj * (1.0 - vk)
                    out["C_n"] += m * (1.0 - vj)
    keep = (mask != 0).astype(np.float64)
    for k in list(out):
        out[k] = out[k] * keep
    out["Atot"] = atot
    return out


@dataclass
class CCSystem(System):
    def source(self, grads) -> np.ndarray:
        return source_cc(self, grads)


def assemble_cc(mask, spacing, n_gl=24) -> CCSystem:
    """[W^{n+1}] = I - W^{n+1} and [W^n] = W^n (diagonal w_C^n) over the data
    cells, numbered in storage order, with w_j^i = A_j^i / A_tot."""
    mask = np.asarray(mask)
    spacing = tuple(float(s) for s in spacing)
    cnt = cc_counters(mask, spacing, n_gl)
    Atot = cnt["Atot"]
    valid = mask != 0
    index = np.full(mask.shape, -1, dtype=np.int64)
    n = int(valid.sum())
    index[valid] = np.arange(n)
    pad = np.pad(index, 1, constant_values=-1)
    ny, nx = mask.shape
    rows, cols, mv = [np.arange(n)], [np.arange(n)], [np.ones(n)]
    nrows, ncols, nv = [np.arange(n)], [np.arange(n)], [cnt["C_n"][valid] / Atot]
    nbr = {}
    for name, ox, oy in CC_DIRECTIONS:
        jidx = pad[1 + oy: 1 + oy + ny, 1 + ox: 1 + ox + nx]
        pair = valid & (jidx >= 0)
        r, c = index[pair], jidx[pair]
        nbr[name] = (r, c)
        rows.append(r)
        cols.append(c)
        mv.append(-cnt[(name, "np1")][pair] / Atot)
        nrows.append(r)
        ncols.append(c)
        nv.append(cnt[(name, "n")][pair] / Atot)
    M = sp.csr_matrix((np.concatenate(mv), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    N = sp.csr_matrix((np.concatenate(nv), (np.concatenate(nrows), np.concatenate(ncols))), shape=(n, n))
    consts = {"Atot": Atot}
    return CCSystem(2, (nx, ny), spacing, consts, valid, index, cnt, M, N, nbr)


def source_cc(system, grads) -> np.ndarray:
    """S_C = - sum_J Delta_J . (w_J^{n+1} + w_J^n) (f(J) + f(C)) / 2 over the
    8 neighbours, Delta_J . f = dx_J h_x f_x + dy_J h_y f_y."""
    Atot = system.consts["Atot"]
    valid = system.valid
    gx, gy = (np.asarray(g, dtype=np.float64)[valid] for g in grads[:2])
    hx, hy = system.spacing
    S = np.zeros(system.n)
    for name, ox, oy in CC_DIRECTIONS:
        r, c = system.nbr[name]
        if r.size == 0:
            continue
        w = (system.counters[(name, "np1")][valid][r] + system.counters[(name, "n")][valid][r]) / Atot
        step = ox * hx * 0.5 * (gx[c] + gx[r]) + oy * hy * 0.5 * (gy[c] + gy[r])
        np.add.at(S, r, -w * step)
    return S
