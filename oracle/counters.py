"""Per-cell ray counters A_j^i of the face-crossing scheme for any mask.

Definitions followed (Section "Weight Computation for Arbitrary Boundary
Shapes"):

* b_j = 1 where cell j holds no data, b~_j = 1 - b_j; a cell outside the grid
  counts as missing (the corner cell of the appendix example has
  A_C^n = 4 Delta, Table tab:Coeffs).
* 2-D, Eqs. AEnp1 / AEn and ANnp1 / ANn:
      A_E^{n+1} = b~_E [c_xy (b~_ES + b~_EN) + c_xx b~_EE]
      A_E^{n}   = b~_E [c_xy (b_ES  + b_EN ) + c_xx b_EE ]
  with E <-> W swapped for the west face and c_xx -> c_yy for north/south.
* 3-D (the A_N equations of the 3-D section and the permutation rule stated
  after them): the face neighbour's laterals along each of the two other axes
  carry the dihedral constant of that axis pair, the far cell carries c_jj.
* Eq. Acn: A_C^n = sum over faces of b_J times the face total
  (2-D: 2 dy (b_E + b_W) + 2 dx (b_N + b_S); 3-D: pi * area).
* Eq. wcnp1: A_C^{n+1} = 0.

Arrays are in storage order (x fastest), so grid axis a is array axis
ndim - 1 - a.  Values at masked cells are set to zero (they own no equation).
"""

from __future__ import annotations

import numpy as np

from .constants import as_array, constants

# (name, grid axis, sign): E = +x, W = -x, N = +y, S = -y, F = +z, B = -z
DIRECTIONS = (("E", 0, +1), ("W", 0, -1), ("N", 1, +1), ("S", 1, -1), ("F", 2, +1), ("B", 2, -1))


def directions(ndim: int):
    return DIRECTIONS[: 2 * ndim]


class _Shifter:
    """Reads b~ at (cell + offset) for every cell at once; outside = 0."""

    PAD = 2

    def __init__(self, mask: np.ndarray):
        self.ndim = mask.ndim
        self.shape = mask.shape
        self.padded = np.pad(mask != 0, self.PAD, constant_values=False).astype(np.float64)

    def valid(self, offset):
        sl = []
        for arr_ax in range(self.ndim):
            a = self.ndim - 1 - arr_ax
            o = offset[a]
            sl.append(slice(self.PAD + o, self.PAD + o + self.shape[arr_ax]))
        return self.padded[tuple(sl)]


def ray_counters(mask: np.ndarray, spacing, consts: dict | None = None) -> dict:
    """Return {'C_n': A_C^n, 'C_np1': A_C^{n+1}, (d, 'np1'): A_d^{n+1},
    (d, 'n'): A_d^n} for every face direction d, as storage-order arrays."""
    ndim = mask.ndim
    if consts is None:
        consts = constants(spacing)
    c = as_array(consts, ndim)
    face = consts["face"]
    sh = _Shifter(mask)
    own = sh.valid((0, 0, 0))
    out = {"C_np1": np.zeros(mask.shape), "C_n": np.zeros(mask.shape)}
    for name, a, s in directions(ndim):
        J = [0, 0, 0]
        J[a] = s
        bt_J = sh.valid(J)
        lat_np1 = np.zeros(mask.shape)
        lat_n = np.zeros(mask.shape)
        for k in range(ndim):
            if k == a:
                continue
            for t in (+1, -1):
                off = list(J)
                off[k] += t
                v = sh.valid(off)
                lat_np1 += c[a, k] * v
                lat_n += c[a, k] * (1.0 - v)
        far = list(J)
        far[a] += s
        v_far = sh.valid(far)
        out[(name, "np1")] = own * bt_J * (lat_np1 + c[a, a] * v_far)
        out[(name, "n")] = own * bt_J * (lat_n + c[a, a] * (1.0 - v_far))
        out["C_n"] += own * (1.0 - bt_J) * face[a]
    return out
