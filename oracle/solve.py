"""Algorithm 1 and its fixed point, in FP64 on the CPU.

Route O1 -- Algorithm 1 as stated: start from {P^0} = 0 (or a given guess),
solve Eq. MatrixEquation for {P^{n+1}} exactly (scipy's sparse LU stands in
for Matlab's backslash, which the paper's CPU code uses), evaluate the
momentum residual of Eq. ResidualMomentum, and repeat while it exceeds the
threshold.

Route O2 -- the fixed point.  At convergence {P^{n+1}} = {P^n} = P, so
(M - N) P = S.  For every valid cell the counters of a face add up to the
face total and all counters add up to A_tot (Eq. Atot2D and its 3-D analogue,
and the remark after the appendix cell-1 example), which makes M - N a
symmetric, zero-row-sum operator: P is defined up to one constant per
connected group of valid cells.  O2 solves it with one cell per group
pinned (least squares in the rounding-level inconsistency), then applies the
gauge.

Gauge: the paper fixes the free constant with one reference point (Sections
on the PIV and SPIV examples).  Here the mean over every face-connected group
of valid cells is removed instead, so that results can be compared cell by
cell; a cell with no valid face neighbour forms its own group and gets 0.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

from .system import System


def residual_momentum(system: System, S, P) -> float:
    """Eq. ResidualMomentum: ||[W^{n+1}]P - [W^n]P - S|| / ||S||."""
    r = system.M @ P - system.N @ P - S
    nS = np.linalg.norm(S)
    return float(np.linalg.norm(r) / nS) if nS > 0 else float(np.linalg.norm(r))


def residual_pressure(P_new, P_old) -> float:
    """Eq. ResidualPressure: ||P^{n+1} - P^n|| / ||P^{n+1}||."""
    d = np.linalg.norm(P_new)
    return float(np.linalg.norm(P_new - P_old) / d) if d > 0 else 0.0


def components(system: System):
    """Face-connected groups of valid cells: (count, label per unknown)."""
    n = system.n
    rows, cols = [], []
    for r, c in system.nbr.values():
        rows.append(r)
        cols.append(c)
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = cols = np.zeros(0, dtype=np.int64)
    A = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    return connected_components(A, directed=False)


def gauge(system: System, P) -> np.ndarray:
    """Remove the mean of P over each connected group of valid cells."""
    k, lab = components(system)
    P = np.asarray(P, dtype=np.float64)
    sums = np.bincount(lab, weights=P, minlength=k)
    cnts = np.bincount(lab, minlength=k)
    return P - (sums / cnts)[lab]


@dataclass
class OuterResult:
    P: np.ndarray
    outer: int
    eps_R: list = field(default_factory=list)
    eps_P: list = field(default_factory=list)
    converged: bool = False


def outer_iteration(system: System, S, tol: float, max_iter: int, P0=None) -> OuterResult:
    """Route O1: Algorithm 1 with an exact inner solve.

    The loop stops as soon as the momentum residual of the current iterate is
    at or below ``tol``; ``outer`` counts the solves of Eq. MatrixEquation."""
    n = system.n
    P = np.zeros(n) if P0 is None else np.array(P0, dtype=np.float64)
    lu = spla.splu(system.M.tocsc())
    res = OuterResult(P, 0)
    eps = residual_momentum(system, S, P)
    res.eps_R.append(eps)
    while eps > tol and res.outer < max_iter:
        P_new = lu.solve(system.N @ P + S)
        res.eps_P.append(residual_pressure(P_new, P))
        P = P_new
        res.outer += 1
        eps = residual_momentum(system, S, P)
        res.eps_R.append(eps)
    res.P = P
    res.converged = eps <= tol
    return res


def fixed_point(system: System, S) -> np.ndarray:
    """Route O2: (M - N) P = S, gauged.

    The fixed point is defined up to one constant per connected group.  An
    assembled L = M - N has column sums of ~1e-15 instead of 0, so in
    floating point the equations are inconsistent at rounding level, and
    the answer wanted is the least-squares one, whose residual is a
    constant lam_g over each group.  With one cell per group pinned (sparse
    LU of the rest), the equations of the other cells are met with S - lam
    and the pinned cell's equation takes the inconsistency; taking lam_g as
    the mean residual over the group and solving again moves that residual
    evenly onto the group (left in one equation, it acts as a point
    source)."""
    L = system.L.tocsr()
    k, lab = components(system)
    n = system.n
    S = np.asarray(S, dtype=np.float64)
    _, first = np.unique(lab, return_index=True)
    keep = np.ones(n, dtype=bool)
    keep[first] = False
    P = np.zeros(n)
    if keep.any():
        lu = spla.splu(L[keep][:, keep].tocsc())
        cnt = np.bincount(lab, minlength=k)
        lam = np.zeros(k)
        for _ in range(3):
            P[keep] = lu.solve((S - lam[lab])[keep])
            lam = np.bincount(lab, weights=S - L @ P, minlength=k) / cnt
    return gauge(system, P)
