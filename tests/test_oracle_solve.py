"""Pins of the oracle's Algorithm-1 iteration (O1) and fixed-point solve (O2)
against exact solutions, invariances and the paper's stated behaviour."""

import numpy as np
import pytest
import torch

import synth
from oracle.solve import (components, fixed_point, fixed_point_cg, gauge, outer_iteration,
                          residual_momentum)
from oracle.system import assemble


def _np(t):
    return t.detach().cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t)


def _disk_mask(dims, seed, frac):
    return _np(synth.disk_mask(dims, seed, frac=frac, rmin=0.08, rmax=0.2))


def _rel_maxabs(a, b):
    rms = np.sqrt(np.mean(b**2))
    return np.abs(a - b).max() / rms


@pytest.mark.parametrize("dims,spacing", [((13, 10), (0.7, 1.1)), ((7, 6, 5), (1.0, 0.6, 1.4))])
def test_quadratic_pressure_recovered_exactly(dims, spacing):
    # A degree-2 field makes the trapezoid face rule exact, so the gradient is
    # consistent and both routes must return the field up to a constant.
    P, g, sp = synth.quadratic(dims, seed=4, spacing=spacing)
    mask = _disk_mask(dims, 3, 0.15)
    sys_ = assemble(mask, sp)
    S = sys_.source([_np(x) for x in g])
    truth = gauge(sys_, sys_.from_grid(_np(P)))
    p2 = fixed_point(sys_, S)
    assert _rel_maxabs(p2, truth) < 1e-11
    res = outer_iteration(sys_, S, tol=1e-13, max_iter=20000)
    assert res.converged
    assert _rel_maxabs(gauge(sys_, res.P), truth) < 1e-10


@pytest.mark.parametrize("dims,spacing", [((17, 12), (1.0, 0.6)), ((6, 7, 5), (1.0, 0.7, 1.9))])
def test_outer_iteration_reaches_fixed_point(dims, spacing):
    rng = np.random.default_rng(2)
    mask = _disk_mask(dims, 5, 0.2)
    sys_ = assemble(mask, spacing)
    g = [rng.normal(size=mask.shape) for _ in dims]   # far from curl-free
    S = sys_.source(g)
    res = outer_iteration(sys_, S, tol=1e-13, max_iter=50000)
    assert res.converged
    p2 = fixed_point(sys_, S)
    assert _rel_maxabs(gauge(sys_, res.P), p2) < 1e-10
    # Appendix: the iteration was never seen to diverge from P^0 = 0
    eps = np.array(res.eps_R)
    assert eps[0] == pytest.approx(1.0)
    assert np.all(eps <= 1.0 + 1e-12)


def test_constant_offset_invariance():
    dims = (15, 11)
    w = synth.random_small(7, 2, dims)
    sys_ = assemble(_np(w.mask), w.spacing)
    S = sys_.source([_np(x) for x in w.grads])
    rng = np.random.default_rng(0)
    P0 = rng.normal(size=sys_.n)
    a = outer_iteration(sys_, S, tol=1e-7, max_iter=5000, P0=P0)
    b = outer_iteration(sys_, S, tol=1e-7, max_iter=5000, P0=P0 + 3.25)
    assert a.outer == b.outer
    # identical step by step up to the rounding of (M - N) P at |P| ~ 4
    assert np.allclose(a.eps_R, b.eps_R, rtol=1e-5, atol=0)
    assert np.abs(gauge(sys_, a.P) - gauge(sys_, b.P)).max() < 1e-10
    # a converged field shifted by a constant needs no iteration at all
    p2 = fixed_point(sys_, S)
    c = outer_iteration(sys_, S, tol=1e-9, max_iter=10, P0=p2 + 17.0)
    assert c.outer == 0


def test_scale_invariance():
    # (spacing, gradient) -> (alpha spacing, gradient / alpha) is the same problem
    dims = (12, 9)
    w = synth.random_small(8, 2, dims)
    g = [_np(x) for x in w.grads]
    m = _np(w.mask)
    p1 = fixed_point(assemble(m, w.spacing), assemble(m, w.spacing).source(g))
    alpha = 3.7
    sp2 = tuple(alpha * s for s in w.spacing)
    sys2 = assemble(m, sp2)
    p2 = fixed_point(sys2, sys2.source([x / alpha for x in g]))
    assert _rel_maxabs(p2, p1) < 1e-12


def test_first_moment_invariant():
    # With an exact inner solve 1^T [W^{n+1}] P^n does not change from one
    # sweep to the next (columns of M - N sum to zero and S sums to zero).
    dims = (14, 9)
    w = synth.random_small(9, 2, dims)
    sys_ = assemble(_np(w.mask), w.spacing)
    S = sys_.source([_np(x) for x in w.grads])
    P = np.zeros(sys_.n)
    import scipy.sparse.linalg as spla
    lu = spla.splu(sys_.M.tocsc())
    scale = np.abs(S).sum()
    for _ in range(25):
        P = lu.solve(sys_.N @ P + S)
        assert abs((sys_.M @ P).sum()) < 1e-12 * scale


def test_isolated_cells_and_components():
    m = np.ones((9, 12), np.uint8)
    m[:, 5] = 0          # splits the grid into two groups
    m[2, 8] = 1
    m[1, 8] = 0
    m[3, 8] = 0
    m[2, 7] = 0
    m[2, 9] = 0          # cell (y=2, x=8) has no face neighbour with data
    sys_ = assemble(m, (1.0, 1.0))
    k, lab = components(sys_)
    assert k == 3
    rng = np.random.default_rng(1)
    S = sys_.source([rng.normal(size=m.shape), rng.normal(size=m.shape)])
    P = fixed_point(sys_, S)
    iso = sys_.index[2, 8]
    assert P[iso] == 0.0
    for c in range(k):
        assert abs(P[lab == c].mean()) < 1e-13
    assert residual_momentum(sys_, S, P) < 1e-12


def test_second_order_convergence():
    # Smooth field, no noise: error against the analytic pressure falls as h^2.
    errs = []
    for n in (16, 32, 64):
        P, g, sp = synth.gaussian_blobs((n, n), seed=12, nblobs=4, sigma_range=(0.15, 0.25))
        sys_ = assemble(np.ones((n, n), np.uint8), sp)
        p = fixed_point(sys_, sys_.source([_np(x) for x in g]))
        t = gauge(sys_, sys_.from_grid(_np(P)))
        errs.append(np.sqrt(np.mean((p - t) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7


def test_residual_decay_rates_agree():
    # The momentum residual and the pressure-update residual decay at the same
    # rate (Section "Method Convergence").
    w = synth.config_sin64(n=24)
    sys_ = assemble(np.ones((24, 24), np.uint8), w.spacing)
    S = sys_.source([_np(x) for x in w.grads])
    res = outer_iteration(sys_, S, tol=1e-11, max_iter=5000)
    eR = np.array(res.eps_R[1:])
    eP = np.array(res.eps_P)
    k = len(eP) // 2
    rate_R = (eR[-1] / eR[k]) ** (1.0 / (len(eR) - 1 - k))
    rate_P = (eP[-1] / eP[k]) ** (1.0 / (len(eP) - 1 - k))
    assert rate_R == pytest.approx(rate_P, rel=1e-3)


def test_taylor_vortex_accuracy():
    # The paper's synthetic case (Section "Taylor Vortex (2D)"): 101^2 grid on
    # [-3, 3]^2, exact gradient, no noise: the integrated field matches the
    # analytic pressure to well under 1 % of the peak suction.
    P, g, sp = synth.taylor_vortex((101, 101), t=0.1)
    sys_ = assemble(np.ones((101, 101), np.uint8), sp)
    p = fixed_point(sys_, sys_.source([_np(x) for x in g]))
    t = gauge(sys_, sys_.from_grid(_np(P)))
    peak = np.abs(_np(P)).max()
    assert np.sqrt(np.mean((p - t) ** 2)) / peak < 2e-3


def test_fixed_point_is_least_squares_in_the_group_constants():
    """(M - N) has zero column sums, so a constant added to S over one group
    has no solution; the oracle takes the least-squares answer, which is the
    solution for S with that constant removed, and it spreads the residual
    evenly over the group instead of leaving it in one pinned cell."""
    m = np.ones((14, 17), np.uint8)
    m[:, 8] = 0                                  # two groups
    sys_ = assemble(m, (0.9, 1.2))
    k, lab = components(sys_)
    assert k == 2
    rng = np.random.default_rng(4)
    S = sys_.source([rng.normal(size=m.shape), rng.normal(size=m.shape)])
    P = fixed_point(sys_, S)
    shift = np.where(lab == 0, 1e-6, -3e-6)      # one constant per group
    Q = fixed_point(sys_, S + shift)
    assert np.abs(Q - P).max() < 1e-12 * np.abs(P).max()
    r = S + shift - sys_.L @ Q
    for c in range(k):
        rc = r[lab == c]
        assert np.abs(rc - rc.mean()).max() < 1e-12 * np.abs(S).max()
        assert abs(rc.mean() - shift[lab == c][0]) < 1e-12


@pytest.mark.parametrize("dims,mask_frac,seed", [((29, 23), 0.15, 21), ((14, 11, 9), 0.12, 22),
                                                 ((40, 9, 7), 0.0, 23)])
def test_fixed_point_cg_matches_the_direct_route(dims, mask_frac, seed):
    """Route O2-CG against route O2 (sparse LU with pinned cells): two
    different algorithms for the same fixed point, on masked grids with
    several groups, isolated cells and anisotropic spacing."""
    w = synth.random_small(seed, len(dims), dims, mask_frac=mask_frac)
    mask = np.ones(tuple(reversed(dims)), np.uint8) if w.mask is None else _np(w.mask)
    sys_ = assemble(mask, w.spacing)
    S = sys_.source([_np(x) for x in w.grads])
    ref = fixed_point(sys_, S)
    res = fixed_point_cg(sys_, S, rtol=1e-14)
    assert res.converged and res.rel_residual < 1e-12
    assert _rel_maxabs(res.P, ref) < 1e-11
    k, lab = components(sys_)
    for c in range(k):
        assert abs(res.P[lab == c].mean()) < 1e-13 * np.abs(ref).max()


def test_fixed_point_cg_exact_on_quadratic_fields():
    P, g, sp = synth.quadratic((11, 9, 8), seed=6, spacing=(0.8, 1.3, 1.0))
    mask = _disk_mask((11, 9, 8), 4, 0.12)
    sys_ = assemble(mask, sp)
    truth = gauge(sys_, sys_.from_grid(_np(P)))
    res = fixed_point_cg(sys_, sys_.source([_np(x) for x in g]), rtol=1e-14)
    assert _rel_maxabs(res.P, truth) < 1e-11


def test_fixed_point_cg_ignores_group_constants_in_the_source():
    # the projection onto the operator's range: a constant per group added to
    # S changes nothing (the least-squares reading of route O2)
    m = np.ones((12, 15), np.uint8)
    m[:, 6] = 0
    sys_ = assemble(m, (1.0, 0.7))
    k, lab = components(sys_)
    rng = np.random.default_rng(8)
    S = sys_.source([rng.normal(size=m.shape), rng.normal(size=m.shape)])
    a = fixed_point_cg(sys_, S, rtol=1e-14).P
    b = fixed_point_cg(sys_, S + np.where(lab == 0, 2e-3, -5e-3), rtol=1e-14).P
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()


@pytest.mark.parametrize("dims,mask_frac", [((16, 13), 0.15), ((9, 8, 7), 0.1)])
def test_one_outer_step_from_a_start_exact_where_w_n_reads(dims, mask_frac):
    """Eq. MatrixEquation reads P^n only through [W^n], whose off-diagonal
    w_j^n is non-zero only where a ray starts at J (a cell next to a missing
    or out-of-grid cell) and whose diagonal w_C^n only where C itself has a
    face without data.  So one exact outer step from any P^0 that equals the
    fixed point on the cells [W^n] reads (its non-zero columns) lands on the
    fixed point, whatever P^0 holds elsewhere, while an error on one of those
    cells is carried on."""
    w = synth.random_small(31, len(dims), dims, mask_frac=mask_frac)
    sys_ = assemble(_np(w.mask), w.spacing)
    S = sys_.source([_np(x) for x in w.grads])
    star = fixed_point(sys_, S)
    Nc = sys_.N.tocsc(copy=True)
    Nc.eliminate_zeros()
    read = np.diff(Nc.indptr) > 0
    # the cells [W^n] reads are exactly those with a face neighbour without data
    face_gap = np.zeros(sys_.n, bool)
    for name, _, _ in __import__("oracle.counters", fromlist=["directions"]).directions(len(dims)):
        r, _ = sys_.nbr[name]
        has = np.zeros(sys_.n, bool)
        has[r] = True
        face_gap |= ~has
    assert np.array_equal(read, face_gap)
    assert 0 < read.sum() < sys_.n
    rng = np.random.default_rng(3)
    P0 = np.where(read, star + 0.75, rng.normal(size=sys_.n) * 10)
    res = outer_iteration(sys_, S, tol=0.0, max_iter=1, P0=P0)
    assert _rel_maxabs(gauge(sys_, res.P), star) < 1e-10
    assert residual_momentum(sys_, S, res.P) < 1e-11
    # one wrong value on a cell that [W^n] reads is not undone in one step
    P0[np.flatnonzero(read)[read.sum() // 2]] += 1.0
    res = outer_iteration(sys_, S, tol=0.0, max_iter=1, P0=P0)
    assert residual_momentum(sys_, S, res.P) > 1e-6
