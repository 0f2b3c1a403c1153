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

Route O2-CG -- the same fixed point for grids too large for a sparse LU:
textbook conjugate gradients in FP64 on the assembled M - N.  The source is
first projected onto the operator's range (its mean over every connected
group removed, the least-squares reading of the rounding-level
inconsistency described above), so the system is consistent and CG from 0
stays in the range; the result is then gauged.

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


@dataclass
class CgResult:
    P: np.ndarray
    iters: int
    rel_residual: float      # ||b - L P|| / ||b||, recomputed from P at the end
    converged: bool


def fixed_point_cg(system: System, S, rtol: float = 1e-13, max_iter: int = 200000) -> CgResult:
    """Route O2-CG: (M - N) P = S by plain conjugate gradients in FP64, gauged.

    L = M - N is symmetric positive semi-definite with one zero eigenvalue per
    connected group (the constants).  b = S minus its mean over each group
    lies in L's range, so CG from P = 0 solves L P = b; the stopping test is
    on the recursively updated residual, ||r|| <= rtol ||b||.  One sparse
    product, two dot products and three vector updates per iteration, no
    preconditioner."""
    L = system.L.tocsr()
    k, lab = components(system)
    S = np.asarray(S, dtype=np.float64)
    cnt = np.bincount(lab, minlength=k)
    b = S - (np.bincount(lab, weights=S, minlength=k) / cnt)[lab]
    nb = float(np.linalg.norm(b))
    P = np.zeros(system.n)
    if nb == 0.0:
        return CgResult(gauge(system, P), 0, 0.0, True)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    it = 0
    while it < max_iter and np.sqrt(rr) > rtol * nb:
        q = L @ p
        alpha = rr / float(p @ q)
        P += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    rel = float(np.linalg.norm(b - L @ P) / nb)
    return CgResult(gauge(system, P), it, rel, np.sqrt(rr) <= rtol * nb)
