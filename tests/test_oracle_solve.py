"""Pins of the oracle's Algorithm-1 iteration (O1) and fixed-point solve (O2)
against exact solutions, invariances and the paper's stated behaviour."""

import numpy as np
import pytest
import torch

import synth
from oracle.solve import (components, fixed_point, gauge, outer_iteration,
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
