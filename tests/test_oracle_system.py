"""Pins of the oracle's counters, matrices and source vector against the
paper's worked 3x3 example, invariants it states, and traced rays."""

import math

import numpy as np
import pytest

from oracle.constants import constants_2d
from oracle.counters import ray_counters
from oracle.rays import ray_counters_bruteforce
from oracle.system import assemble
from conftest import read_golden, paper_cell_to_storage



def _eval_token(tok, c, D=1.0):
    total = 0.0
    for term in tok.split("+"):
        term = term.strip()
        if term == "0":
            continue
        m = 1.0
        i = 0
        while i < len(term) and term[i].isdigit():
            i += 1
        if i:
            m = float(term[:i])
        sym = term[i:]
        if sym == "D":
            total += m * D
        else:
            total += m * c[sym[1:]]
    return total


def _appendix_counters(corrected=True):
    """Table tab:Coeffs as printed, with the listed errata applied unless
    ``corrected`` is False."""
    c = constants_2d(1.0, 1.0)["c"]
    table = {}
    errata = []
    for row in read_golden("appendix_3x3_counters.txt"):
        if row[0] == "ERRATUM":
            errata.append((row[1], int(row[2]), _eval_token(row[3], c)))
            continue
        table[row[0]] = [_eval_token(t, c) for t in row[1:]]
    if corrected:
        for name, k, v in errata:
            table[name][k - 1] = v
    return table


def test_appendix_erratum_is_a_swap_restoring_mirror_symmetry():
    printed = _appendix_counters(corrected=False)
    fixed = _appendix_counters(corrected=True)
    changed = [(n, k) for n in printed for k in range(9) if printed[n][k] != fixed[n][k]]
    assert sorted(changed) == [("N_n", 3), ("N_np1", 3)]
    assert printed["N_n"][3] == fixed["N_np1"][3] and printed["N_np1"][3] == fixed["N_n"][3]
    # corrected cell 4 looks the same north and south, and equals its mirror cell 6
    for it in ("n", "np1"):
        assert fixed["N_" + it][3] == fixed["S_" + it][3] == fixed["N_" + it][5] == fixed["S_" + it][5]


def test_appendix_table_of_counters():
    table = _appendix_counters()
    cnt = ray_counters(np.ones((3, 3), np.uint8), (1.0, 1.0))
    for name, vals in table.items():
        d, it = name.split("_")
        key = "C_" + it if d == "C" else (d, it)
        for k, v in enumerate(vals, start=1):
            y, x = paper_cell_to_storage(k)
            assert cnt[key][y, x] == pytest.approx(v, abs=1e-14), (name, k)


def test_appendix_counters_sum_to_atot():
    # remark after the cell-1 example: all ten counters add up to A_tot = 8 D
    table = _appendix_counters()
    for k in range(9):
        assert sum(v[k] for v in table.values()) == pytest.approx(8.0, abs=1e-14)


def _storage_index(k):
    y, x = paper_cell_to_storage(k)
    return y * 3 + x


def test_appendix_matrices():
    # Eq. GiantMatrix: pentadiagonal pattern; entries w = A / A_tot with
    # [W^{n+1}] = I - W^{n+1} and [W^n] = W^n, diagonal of [W^n] = w_C^n.
    table = _appendix_counters()
    sys_ = assemble(np.ones((3, 3), np.uint8), (1.0, 1.0))
    M = sys_.M.toarray()
    N = sys_.N.toarray()
    pattern = {int(r[0]): [int(v) for v in r[1:]] for r in read_golden("appendix_3x3_pattern.txt")}
    for k, cols in pattern.items():
        i = _storage_index(k)
        nz_M = sorted(j for j in range(9) if M[i, j] != 0)
        assert nz_M == sorted(_storage_index(c) for c in cols)
        nz_N = set(j for j in range(9) if N[i, j] != 0)
        assert nz_N <= set(_storage_index(c) for c in cols)
    step = {"E": (0, 1), "W": (0, -1), "N": (1, 0), "S": (-1, 0)}
    for k in range(1, 10):
        i = _storage_index(k)
        y, x = paper_cell_to_storage(k)
        assert M[i, i] == pytest.approx(1.0 - table["C_np1"][k - 1] / 8.0, abs=1e-15)
        assert N[i, i] == pytest.approx(table["C_n"][k - 1] / 8.0, abs=1e-15)
        for d, (dy, dx) in step.items():
            yy, xx = y + dy, x + dx
            if not (0 <= yy < 3 and 0 <= xx < 3):
                continue
            j = yy * 3 + xx
            assert M[i, j] == pytest.approx(-table[d + "_np1"][k - 1] / 8.0, abs=1e-15)
            assert N[i, j] == pytest.approx(table[d + "_n"][k - 1] / 8.0, abs=1e-15)
    # the operator is not symmetric near the boundary: cell 1 sees cell 2 with
    # c_xy + c_xx, cell 2 sees cell 1 with c_xy (Table tab:Coeffs)
    assert M[_storage_index(1), _storage_index(2)] != pytest.approx(M[_storage_index(2), _storage_index(1)])


def test_appendix_source_rows():
    rng = np.random.default_rng(0)
    fx = rng.normal(size=(3, 3))
    fy = rng.normal(size=(3, 3))
    for D in (1.0, 0.37):
        sys_ = assemble(np.ones((3, 3), np.uint8), (D, D))
        S = sys_.source([fx, fy])
        for row in read_golden("appendix_3x3_source.txt"):
            k = int(row[0][1:])
            acc = 0.0
            for q in range(1, len(row), 3):
                comp, cell, coef = row[q], int(row[q + 1]), float(row[q + 2])
                y, x = paper_cell_to_storage(cell)
                acc += coef * (fx if comp == "fx" else fy)[y, x]
            assert S[_storage_index(k)] == pytest.approx(-(D / 8.0) * acc, abs=1e-14)


def test_appendix_dependency_footprint():
    # Appendix: if cell 1 held NaN, the counters of cells 2, 3, 4, 5 and 7
    # would change and all other cells would be unaffected.
    full = ray_counters(np.ones((3, 3), np.uint8), (1.0, 1.0))
    m = np.ones((3, 3), np.uint8)
    y1, x1 = paper_cell_to_storage(1)
    m[y1, x1] = 0
    holed = ray_counters(m, (1.0, 1.0))
    changed = set()
    for key in full:
        diff = np.abs(full[key] - holed[key]) > 0
        for k in range(2, 10):
            y, x = paper_cell_to_storage(k)
            if diff[y, x]:
                changed.add(k)
    assert changed == {2, 3, 4, 5, 7}


def _random_mask(shape, seed, frac):
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=shape) > frac).astype(np.uint8)


CASES = [((7, 9), (1.0, 0.6)), ((5, 6, 4), (1.0, 0.7, 1.9)), ((6, 5, 5), (0.5, 0.5, 0.5))]


@pytest.mark.parametrize("shape,spacing", CASES)
def test_counters_sum_and_face_totals(shape, spacing):
    mask = _random_mask(shape, 3, 0.3)
    sys_ = assemble(mask, spacing)
    cnt = sys_.counters
    valid = mask != 0
    total = cnt["C_n"] + cnt["C_np1"]
    ndim = mask.ndim
    for key, arr in cnt.items():
        if isinstance(key, tuple):
            total = total + arr
    assert np.allclose(total[valid], sys_.consts["Atot"], rtol=0, atol=1e-12)
    # A_j^{n+1} + A_j^n is the face total when J holds data, else zero
    from oracle.counters import directions
    for name, a, s in directions(ndim):
        both = cnt[(name, "np1")] + cnt[(name, "n")]
        vals = np.unique(np.round(both[valid], 12))
        assert set(vals.tolist()) <= {0.0, round(sys_.consts["face"][a], 12)}


@pytest.mark.parametrize("shape,spacing", CASES)
def test_fixed_point_operator_is_a_laplacian(shape, spacing):
    mask = _random_mask(shape, 5, 0.25)
    sys_ = assemble(mask, spacing)
    L = sys_.L.toarray()
    assert np.allclose(L, L.T, atol=1e-14)
    assert np.allclose(L.sum(axis=1), 0.0, atol=1e-14)
    off = L - np.diag(np.diag(L))
    assert (off <= 1e-15).all()
    # the source vector sums to zero: face terms cancel pairwise
    rng = np.random.default_rng(1)
    g = [rng.normal(size=mask.shape) for _ in range(mask.ndim)]
    S = sys_.source(g)
    assert abs(S.sum()) < 1e-12 * max(1.0, np.abs(S).sum())


@pytest.mark.parametrize("shape,spacing", [((6, 7), (1.0, 0.6)), ((5, 4), (0.7, 1.3))])
def test_counters_match_traced_rays_2d(shape, spacing):
    mask = _random_mask(shape, 11, 0.3)
    ref = ray_counters(mask, spacing)
    bf = ray_counters_bruteforce(mask, spacing, n_theta=2000, n_face=2000)
    for key in ref:
        assert np.allclose(bf[key], ref[key], rtol=0, atol=2e-4 * max(spacing)), key


def test_counters_match_traced_rays_3d():
    spacing = (1.0, 0.7, 1.9)
    mask = _random_mask((4, 4, 3), 7, 0.3)
    ref = ray_counters(mask, spacing)
    bf = ray_counters_bruteforce(mask, spacing, n_theta=40, n_face=16)
    for key in ref:
        assert np.allclose(bf[key], ref[key], rtol=0, atol=1.5e-2), key
