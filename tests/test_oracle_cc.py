"""Pins of the cell-centred oracle (oracle/cellcentered.py): closed forms of
the interior counters, counters of explicit rays on a masked grid, mirror
symmetry, the conservation of rays, and exact recovery of quadratic
pressure fields (the trapezoid rule between centres is exact for them)."""

import math

import numpy as np
import pytest

from oracle.cellcentered import CC_DIRECTIONS, assemble_cc, cc_counters
from oracle.rays import cc_counters_bruteforce
from oracle.solve import fixed_point, gauge, outer_iteration

NAMES = [n for n, _, _ in CC_DIRECTIONS]


@pytest.mark.parametrize("sp", [(1.0, 1.0), (0.7, 1.3), (2.0, 0.5)])
def test_interior_counters_closed_forms(sp):
    """An interior cell sees every ray from its 8 neighbours at the current
    sweep.  Integrating the nearest-centre rule by hand (D = |(dx, dy)|):
    a face neighbour along x gets 2 (D - dx), along y 2 (D - dy), a diagonal
    dx + dy - D, and all rays through a cell measure A_tot = 4 D."""
    dx, dy = sp
    D = math.hypot(dx, dy)
    c = cc_counters(np.ones((9, 10), np.uint8), sp)
    ci = (4, 5)
    want = {"E": 2 * (D - dx), "W": 2 * (D - dx), "N": 2 * (D - dy), "S": 2 * (D - dy),
            "NE": dx + dy - D, "NW": dx + dy - D, "SE": dx + dy - D, "SW": dx + dy - D}
    for n in NAMES:
        assert abs(c[(n, "np1")][ci] - want[n]) < 1e-13, n
        assert c[(n, "n")][ci] == 0.0
    assert c["C_n"][ci] == 0.0
    assert abs(c["Atot"] - 4 * D) < 1e-13


def test_counters_match_explicit_rays():
    rng = np.random.default_rng(3)
    m = (rng.random((6, 7)) > 0.25).astype(np.uint8)
    sp = (0.8, 1.1)
    c = cc_counters(m, sp)
    b = cc_counters_bruteforce(m, sp, n_theta=1440, ds=0.005)
    for k in b:
        assert np.abs(b[k] - c[k]).max() < 4e-3, k


def test_every_ray_is_counted_once_and_mirror_symmetry():
    rng = np.random.default_rng(11)
    m = (rng.random((9, 8)) > 0.3).astype(np.uint8)
    sp = (0.9, 1.4)
    c = cc_counters(m, sp)
    tot = c["C_n"] + sum(c[(n, i)] for n in NAMES for i in ("np1", "n"))
    valid = m != 0
    assert np.allclose(tot[valid], c["Atot"], rtol=0, atol=1e-12)
    # mirroring the mask in x swaps east and west
    cm = cc_counters(m[:, ::-1], sp)
    swap = {"E": "W", "W": "E", "N": "N", "S": "S", "NE": "NW", "NW": "NE", "SE": "SW", "SW": "SE"}
    for n in NAMES:
        for i in ("np1", "n"):
            assert np.allclose(cm[(swap[n], i)][:, ::-1], c[(n, i)], atol=1e-13)
    # and transposing the grid (with the spacings) swaps the axes
    ct = cc_counters(m.T, sp[::-1])
    tr = {"E": "N", "W": "S", "N": "E", "S": "W", "NE": "NE", "NW": "SE", "SE": "NW", "SW": "SW"}
    for n in NAMES:
        for i in ("np1", "n"):
            assert np.allclose(ct[(tr[n], i)].T, c[(n, i)], atol=1e-13)


def test_fixed_point_operator_is_a_symmetric_laplacian():
    """For a data neighbour J the two counters add up to the interior value
    of that direction, so M - N = sum_J a_J (P_C - P_J) with constant a_J:
    symmetric, zero row sums."""
    rng = np.random.default_rng(5)
    m = (rng.random((11, 13)) > 0.2).astype(np.uint8)
    s = assemble_cc(m, (0.6, 0.9))
    L = s.L.toarray()
    assert np.allclose(L, L.T, atol=1e-14)
    assert np.allclose(L.sum(axis=1), 0.0, atol=1e-14)
    M = s.M.toarray()
    N = s.N.toarray()
    assert np.allclose((N.sum(axis=1) - (M.sum(axis=1) - 1.0)), 1.0, atol=1e-14)


def test_quadratic_pressure_is_recovered_exactly():
    rng = np.random.default_rng(8)
    ny, nx = 12, 15
    m = (rng.random((ny, nx)) > 0.15).astype(np.uint8)
    sp = (0.7, 1.2)
    y, x = np.meshgrid((np.arange(ny) + 0.5) * sp[1], (np.arange(nx) + 0.5) * sp[0], indexing="ij")
    a = rng.normal(size=6)
    P = a[0] + a[1] * x + a[2] * y + a[3] * x * x + a[4] * x * y + a[5] * y * y
    g = [a[1] + 2 * a[3] * x + a[4] * y, a[2] + a[4] * x + 2 * a[5] * y]
    s = assemble_cc(m, sp)
    S = s.source(g)
    want = gauge(s, s.from_grid(P))
    got = fixed_point(s, S)
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    # Algorithm 1 with exact inner solves approaches the same field
    r = outer_iteration(s, S, tol=1e-12, max_iter=20000)
    assert r.converged
    assert np.abs(gauge(s, r.P) - want).max() < 1e-8 * np.abs(want).max()
