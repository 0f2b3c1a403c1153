"""Explicit sparse assembly of the matrix equation [W^{n+1}]{P^{n+1}} =
[W^n]{P^n} + {S} (Eq. MatrixEquation) for the valid cells of a grid.

Reading of the notation (the appendix matrices of Eq. GiantMatrix):
[W^{n+1}] is the operator M = I - W^{n+1}, whose off-diagonal entries are
-w_j^{n+1} and whose diagonal is 1 - w_C^{n+1} = 1 (Eq. wcnp1); [W^n] is
N = W^n with off-diagonal w_j^n and diagonal w_C^n.  Weights are
w_j^i = A_j^i / A_tot (Eq. weights).  Unknowns are the valid cells, numbered
in storage order (x fastest).

The source vector follows the last sum of Eq. ExplicitEqn_FaceCrossing:
    S_C = - sum_j Delta_j (w_j^{n+1} + w_j^n) (f_j(J) + f_j(C)) / 2
where Delta_j is the signed spacing towards face neighbour J (Delta_E = +dx,
Delta_W = -dx, ...) and f_j the gradient component along that axis.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .constants import constants
from .counters import directions, ray_counters


@dataclass
class System:
    ndim: int
    dims: tuple          # (nx, ny[, nz])
    spacing: tuple
    consts: dict
    valid: np.ndarray    # bool, storage order
    index: np.ndarray    # int64, storage order, unknown number or -1
    counters: dict
    M: sp.csr_matrix     # [W^{n+1}] = I - W^{n+1}
    N: sp.csr_matrix     # [W^n]
    nbr: dict            # direction name -> (rows, cols) of valid (C, J) pairs

    @property
    def n(self) -> int:
        return int(self.valid.sum())

    @property
    def L(self) -> sp.csr_matrix:
        """M - N: the operator whose null residual defines convergence
        (Eq. ResidualMomentum)."""
        return (self.M - self.N).tocsr()

    def to_grid(self, vec, fill=np.nan) -> np.ndarray:
        g = np.full(self.valid.shape, fill, dtype=np.float64)
        g[self.valid] = vec
        return g

    def from_grid(self, arr) -> np.ndarray:
        return np.asarray(arr, dtype=np.float64)[self.valid]

    def source(self, grads) -> np.ndarray:
        """{S} from gradient components given in storage order (FP64 math)."""
        return source(self, grads)


def _shift_index(index, offset, ndim):
    """index[cell + offset] for every cell, -1 outside the grid."""
    pad = np.pad(index, 1, constant_values=-1)
    sl = []
    for arr_ax in range(ndim):
        a = ndim - 1 - arr_ax
        o = offset[a]
        sl.append(slice(1 + o, 1 + o + index.shape[arr_ax]))
    return pad[tuple(sl)]


def assemble(mask, spacing) -> System:
    mask = np.asarray(mask)
    ndim = mask.ndim
    if ndim not in (2, 3):
        raise ValueError("2-D or 3-D grids only")
    spacing = tuple(float(s) for s in spacing)
    consts = constants(spacing)
    valid = mask != 0
    index = np.full(mask.shape, -1, dtype=np.int64)
    n = int(valid.sum())
    index[valid] = np.arange(n)
    cnt = ray_counters(mask, spacing, consts)
    Atot = consts["Atot"]

    rows = [np.arange(n)]
    cols = [np.arange(n)]
    m_vals = [np.ones(n)]                      # 1 - w_C^{n+1}, w_C^{n+1} = 0
    n_rows = [np.arange(n)]
    n_cols = [np.arange(n)]
    n_vals = [cnt["C_n"][valid] / Atot]        # w_C^n
    nbr = {}
    for name, a, s in directions(ndim):
        off = [0, 0, 0]
        off[a] = s
        jidx = _shift_index(index, off, ndim)
        pair = valid & (jidx >= 0)
        r = index[pair]
        cidx = jidx[pair]
        nbr[name] = (r, cidx)
        rows.append(r)
        cols.append(cidx)
        m_vals.append(-cnt[(name, "np1")][pair] / Atot)
        n_rows.append(r)
        n_cols.append(cidx)
        n_vals.append(cnt[(name, "n")][pair] / Atot)
    M = sp.csr_matrix((np.concatenate(m_vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    N = sp.csr_matrix((np.concatenate(n_vals), (np.concatenate(n_rows), np.concatenate(n_cols))),
                      shape=(n, n))
    dims = tuple(reversed(mask.shape))
    return System(ndim, dims, spacing, consts, valid, index, cnt, M, N, nbr)


def source(system: System, grads) -> np.ndarray:
    ndim = system.ndim
    Atot = system.consts["Atot"]
    valid = system.valid
    S = np.zeros(system.n)
    g = [np.asarray(x, dtype=np.float64) for x in grads]
    for name, a, s in directions(ndim):
        r, cidx = system.nbr[name]
        if r.size == 0:
            continue
        fa_C = g[a][valid][r]
        fa_J = g[a][valid][cidx]
        w_sum = (system.counters[(name, "np1")][valid][r] + system.counters[(name, "n")][valid][r]) / Atot
        delta_j = s * system.spacing[a]
        np.add.at(S, r, -delta_j * w_sum * 0.5 * (fa_J + fa_C))
    return S
