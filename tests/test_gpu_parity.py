"""Parity of the HIP library (through its C interface) with the CPU oracle.

Sizes span several strips and segments with ragged tails; results are
compared cell by cell.  Bars: operator applies and the source vector to
rounding; converged pressure max-abs error <= 1e-11 RMS(P) in FP64 mode and
<= 1e-5 RMS(P) in FP32 mode against the oracle's fixed point (route O2).
"""

import numpy as np
import pytest
import torch

import synth
from gpu_common import (DEV, announce, fp32_cases, fp64_cases, np_, oracle_for, rel_maxabs, requires_gpu,
                        small_cases)
from oracle.solve import fixed_point, gauge, outer_iteration, residual_momentum

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = small_cases()


def _plan(w, fp64, **kw):
    import paper_2311_16935_amd as pi

    return pi.Plan(w.dims, w.spacing, mask=w.mask, fp64=fp64, **kw)


def _grads(w, fp64):
    dt = torch.float64 if fp64 else torch.float32
    return [g.to(DEV, dt) for g in w.grads]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_operator_applies(name, make, fp64):
    import paper_2311_16935_amd as pi

    announce("apply", name, fp64)
    w = make()
    sys_ = oracle_for(w)
    plan = _plan(w, fp64)
    rng = np.random.default_rng(5)
    x = np.zeros(sys_.valid.shape)
    x[sys_.valid] = rng.normal(size=sys_.n)
    dt = torch.float64 if fp64 else torch.float32
    xt = torch.tensor(x, dtype=dt, device=DEV)
    xv = x[sys_.valid]
    if not fp64:
        xv = xt.cpu().double().numpy()[sys_.valid]
    refs = {pi.PI_OP_M: sys_.M @ xv, pi.PI_OP_N: sys_.N @ xv, pi.PI_OP_L: sys_.L @ xv}
    for op, ref in refs.items():
        y = np_(plan.apply(op, xt)).astype(np.float64)
        assert np.all(y[~sys_.valid] == 0)
        err = np.abs(y[sys_.valid] - ref).max() / np.abs(ref).max()
        assert err < (1e-14 if fp64 else 2e-6), (op, err)
    plan.close()


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_source(name, make, fp64):
    announce("source", name, fp64)
    w = make()
    sys_ = oracle_for(w)
    plan = _plan(w, fp64)
    g = _grads(w, fp64)
    S = np_(plan.source(g)).astype(np.float64)
    ref = sys_.source([np_(x).astype(np.float64) for x in g])
    assert np.all(S[~sys_.valid] == 0)
    err = np.abs(S[sys_.valid] - ref).max() / np.abs(ref).max()
    assert err < (1e-14 if fp64 else 1e-7), err
    plan.close()


def _converged_fp64(res):
    # stop at 1e-14, or where rounding of the FP64 residual stalls just above it
    return res.status == 0 or (res.status == 4 and res.info["eps_R"] <= 1e-13)


F64 = fp64_cases()
F32 = fp32_cases()


@pytest.mark.parametrize("name,make", F64, ids=[c[0] for c in F64])
def test_solve_fp64_matches_fixed_point(name, make):
    announce("solve-fp64", name)
    w = make()
    sys_ = oracle_for(w)
    plan = _plan(w, True)
    g = _grads(w, True)
    res = plan.solve(g, tol=1e-14, max_iter=300000, check=False)
    assert _converged_fp64(res), res.info
    P = np_(res.P)
    assert np.all(np.isnan(P[~sys_.valid]))
    ref = fixed_point(sys_, sys_.source([np_(x) for x in g]))
    err = rel_maxabs(P[sys_.valid], ref)
    assert err <= 1e-11, err
    plan.close()


@pytest.mark.parametrize("name,make", F32, ids=[c[0] for c in F32])
def test_solve_fp32_matches_fixed_point(name, make):
    announce("solve-fp32", name)
    w = make()
    sys_ = oracle_for(w)
    plan = _plan(w, False)
    g = _grads(w, False)
    res = plan.solve(g, tol=1e-10, max_iter=300000)
    assert res.status == 0, res.info
    P = np_(res.P).astype(np.float64)
    assert np.all(np.isnan(P[~sys_.valid]))
    ref = fixed_point(sys_, sys_.source([np_(x).astype(np.float64) for x in g]))
    err = rel_maxabs(P[sys_.valid], ref)
    assert err <= 1e-5, err
    plan.close()


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_reported_residual_and_gauge(fp64):
    announce("residual", fp64)
    w = synth.random_small(44, 2, (90, 61), mask_frac=0.12)
    sys_ = oracle_for(w)
    plan = _plan(w, fp64)
    g = _grads(w, fp64)
    res = plan.solve(g, tol=1e-7)
    assert res.status == 0 and res.info["eps_R"] <= 1e-7
    P = np_(res.P).astype(np.float64)[sys_.valid]
    S = sys_.source([np_(x).astype(np.float64) for x in g])
    eR = residual_momentum(sys_, S, P)
    if fp64:
        assert eR == pytest.approx(res.info["eps_R"], rel=1e-6)
    else:
        # the returned float field carries its own rounding: its residual is
        # bounded by the FP64 iterate's plus that of rounding the exact
        # fixed point to float
        ref = fixed_point(sys_, S)
        floor = residual_momentum(sys_, S, ref.astype(np.float32).astype(np.float64))
        assert eR <= res.info["eps_R"] + 2.0 * floor, (eR, floor)
    from oracle.solve import components
    k, lab = components(sys_)
    assert res.info["components"] == k
    rms = np.sqrt(np.mean(P**2))
    for c in range(k):
        assert abs(P[lab == c].mean()) < (1e-13 if fp64 else 1e-6) * rms
    plan.close()


def test_bicgstab_inner_solver():
    announce("bicgstab")
    w = synth.random_small(42, 3, (24, 17, 13), mask_frac=0.1)
    sys_ = oracle_for(w)
    plan = _plan(w, True, bicgstab=True, inner_iters=2)
    g = _grads(w, True)
    res = plan.solve(g, tol=1e-14, max_iter=200000, check=False)
    assert _converged_fp64(res), res.info
    ref = fixed_point(sys_, sys_.source([np_(x) for x in g]))
    assert rel_maxabs(np_(res.P)[sys_.valid], ref) <= 1e-11
    plan.close()


def test_exact_inner_solve_follows_algorithm_1():
    # With many inner iterations each outer step is Eq. MatrixEquation solved
    # exactly, so the GPU trajectory follows the oracle's route O1.
    announce("trajectory")
    w = synth.random_small(22, 2, (23, 19), mask_frac=0.1)
    sys_ = oracle_for(w)
    g = _grads(w, True)
    S = sys_.source([np_(x) for x in g])
    ref = outer_iteration(sys_, S, tol=0.0, max_iter=5)
    plan = _plan(w, True, bicgstab=True, inner_iters=200)
    res = plan.solve(g, tol=0.0, max_iter=5)
    assert res.status == 4 and res.info["outer_iters"] == 5
    assert rel_maxabs(np_(res.P)[sys_.valid], gauge(sys_, ref.P)) < 1e-9
    plan.close()


def test_masked_cells_are_ignored():
    announce("masked-nan")
    w = synth.random_small(23, 2, (77, 51), mask_frac=0.15)
    sys_ = oracle_for(w)
    g = _grads(w, True)
    assert any(torch.isnan(x).any() for x in g)   # NaN sits in masked cells
    plan = _plan(w, True)
    a = np_(plan.solve(g, tol=1e-8, max_iter=100000).P)
    g2 = [torch.where(torch.isnan(x), torch.full_like(x, 1e30), x) for x in g]
    b = np_(plan.solve(g2, tol=1e-8, max_iter=100000).P)
    assert np.array_equal(a[sys_.valid], b[sys_.valid])
    plan.close()


def test_error_paths():
    import paper_2311_16935_amd as pi

    announce("errors")
    w = synth.random_small(24, 2, (40, 30), mask_frac=0.1)
    sys_ = oracle_for(w)
    plan = _plan(w, True)
    g = _grads(w, True)
    # a NaN inside a data cell
    bad = [x.clone() for x in g]
    yy, xx = np.argwhere(sys_.valid)[7]
    bad[1][yy, xx] = float("nan")
    r = plan.solve(bad, tol=1e-8, check=False)
    assert r.status == pi.PI_ERR_NONFINITE
    with pytest.raises(pi.PiError):
        plan.source(bad)
    # max_iter reached: last iterate returned, gauged
    r = plan.solve(g, tol=1e-14, max_iter=3, check=False)
    assert r.status == pi.PI_ERR_NOT_CONVERGED and r.info["outer_iters"] == 3
    assert np.isfinite(np_(r.P)[sys_.valid]).all()
    # invalid arguments
    with pytest.raises(pi.PiError):
        pi.pi_plan(2, (0, 5), (1.0, 1.0))
    with pytest.raises(pi.PiError):
        pi.pi_plan(2, (5, 5), (1.0, -1.0))
    with pytest.raises(pi.PiError):
        pi.pi_plan(2, (5, 5), (1.0, 1.0), mask=torch.zeros(5, 5, dtype=torch.uint8))
    rc, _ = pi.pi_solve(plan.handle, g[0], g[1], None, torch.empty_like(g[0]), -1.0, 10)
    assert rc == pi.PI_ERR_INVALID_ARG
    plan.close()


def test_warm_start_and_offsets():
    announce("warm-start")
    w = synth.random_small(25, 2, (60, 45), mask_frac=0.1)
    sys_ = oracle_for(w)
    plan = _plan(w, True)
    g = _grads(w, True)
    base = plan.solve(g, tol=1e-12)
    P0 = base.P.clone()
    P0[torch.isnan(P0)] = 0.0
    P0 += 5.0
    r = plan.solve(g, P=P0, tol=1e-12, warm_start=True)
    assert r.info["outer_iters"] == 0
    assert np.nanmax(np.abs(np_(r.P) - np_(base.P))) < 1e-12 * np.sqrt(np.nanmean(np_(base.P) ** 2))
    # a constant added to the true pressure gives an identical input and result
    zero = [torch.zeros_like(x) for x in g]
    z = plan.solve(zero, tol=1e-9)
    assert z.status == 0 and z.info["outer_iters"] == 0
    assert np.all(np_(z.P)[sys_.valid] == 0)
    plan.close()


def test_batched_matches_single_solves():
    import paper_2311_16935_amd as pi

    announce("batched")
    ws = [synth.random_small(31, 2, (150, 70), mask_frac=0.1),
          synth.random_small(32, 3, (40, 22, 31), mask_frac=0.05),
          synth.random_small(33, 2, (64, 200), mask_frac=0.0),
          synth.random_small(34, 3, (17, 9, 12), anisotropic=False, mask_frac=0.0)]
    for fp64 in (False, True):
        plans = [_plan(w, fp64) for w in ws]
        grads = [_grads(w, fp64) for w in ws]
        tols = [1e-6, 1e-7, 1e-6, 1e-8]
        singles = [p.solve(g, tol=t, max_iter=100000) for p, g, t in zip(plans, grads, tols)]
        rc, Ps, infos = pi.solve_batched(plans, grads, tol=tols, max_iter=100000)
        assert rc == 0
        for s, P, info in zip(singles, Ps, infos):
            assert info["outer_iters"] == s.info["outer_iters"]
            assert torch.equal(torch.nan_to_num(P, nan=7.0), torch.nan_to_num(s.P, nan=7.0))
        # an instance with zero source and a slow one in the same batch
        zero = [torch.zeros_like(x) for x in grads[0]]
        rc, Ps, infos = pi.solve_batched(plans[:2], [zero, grads[1]], tol=[1e-6, 1e-8], max_iter=100000)
        assert rc == 0 and infos[0]["outer_iters"] == 0 and infos[1]["outer_iters"] > 50
        for p in plans:
            p.close()


def test_batched_work_list_drops_finished_instances():
    """A large instance that finishes early (zero source, or a loose
    tolerance) leaves the batched work list: the call rebuilds its tables
    without it, and the instance still running returns exactly what its own
    solve returns."""
    import paper_2311_16935_amd as pi

    announce("batched work list")
    big = synth.random_small(35, 2, (256, 256), mask_frac=0.0)
    small = synth.random_small(36, 3, (24, 17, 13), mask_frac=0.1)
    plans = [_plan(big, False), _plan(small, False)]
    grads = [_grads(big, False), _grads(small, False)]
    single = plans[1].solve(grads[1], tol=1e-9, max_iter=100000)
    for g0, tol0 in (([torch.zeros_like(x) for x in grads[0]], 1e-6), (grads[0], 0.3)):
        rc, Ps, infos = pi.solve_batched(plans, [g0, grads[1]], tol=[tol0, 1e-9], max_iter=100000)
        assert rc == 0, infos
        assert infos[0]["outer_iters"] < infos[1]["outer_iters"]
        assert infos[1]["worklist_rebuilds"] >= 1, infos
        assert infos[1]["outer_iters"] == single.info["outer_iters"]
        assert torch.equal(torch.nan_to_num(Ps[1], nan=7.0), torch.nan_to_num(single.P, nan=7.0))
        # the early instance was gauged and returned like any other
        lone = plans[0].solve(g0, tol=tol0, max_iter=100000)
        assert torch.equal(Ps[0], lone.P)
    for p in plans:
        p.close()


def test_async_solve_matches_the_blocking_one():
    """PI_ASYNC enqueues the solve on the stream and returns at once; after
    a stream sync, P and pi_last_info match the blocking solve exactly, also
    when max_iter stops it first."""
    import paper_2311_16935_amd as pi

    announce("async solve")
    w = synth.random_small(37, 3, (40, 22, 31), mask_frac=0.05)
    for fp64 in (False, True):
        plan = _plan(w, fp64)
        g = _grads(w, fp64)
        for tol, max_iter in ((1e-8, 100000), (1e-12, 40)):
            ref = plan.solve(g, tol=tol, max_iter=max_iter, check=False)
            P = torch.full_like(ref.P, 3.0)
            stream = torch.cuda.current_stream()
            plan.solve_async(g, P, tol=tol, max_iter=max_iter, stream=stream)
            stream.synchronize()
            rc, info = plan.last_info()
            assert rc == ref.status, (rc, ref.status)
            for k in ("outer_iters", "inner_iters_total", "eps_R", "eps_P", "status"):
                assert info[k] == ref.info[k], k
            assert torch.equal(torch.nan_to_num(P, nan=7.0), torch.nan_to_num(ref.P, nan=7.0))
        assert ref.status == pi.PI_ERR_NOT_CONVERGED and ref.info["outer_iters"] == 40
        plan.close()


def test_sin64_config():
    # 64^2, unit spacing, P = sin(2 pi x) cos(2 pi y) with 5 % gradient noise,
    # FP64, solved to eps_R <= 1e-10; against the oracle's Algorithm 1 (exact
    # inner solves) run to the same threshold and its fixed point.
    announce("sin64")
    w = synth.config_sin64()
    sys_ = oracle_for(w)
    g = _grads(w, True)
    S = sys_.source([np_(x) for x in g])
    plan = _plan(w, True)
    r = plan.solve(g, tol=1e-10)
    assert r.status == 0 and r.info["eps_R"] <= 1e-10
    P = np_(r.P)[sys_.valid]
    assert residual_momentum(sys_, S, P) <= 1.01e-10
    o1 = outer_iteration(sys_, S, tol=1e-10, max_iter=100000)
    ref = fixed_point(sys_, S)
    # both sit within their residual-limited distance of the fixed point
    e_gpu = rel_maxabs(P, ref)
    e_o1 = rel_maxabs(gauge(sys_, o1.P), ref)
    assert e_gpu < 1e-7 and e_o1 < 1e-7
    r2 = plan.solve(g, tol=1e-14, max_iter=200000, check=False)
    assert _converged_fp64(r2), r2.info
    assert rel_maxabs(np_(r2.P)[sys_.valid], ref) <= 1e-11
    plan.close()


@pytest.mark.parametrize("ndim,dims", [(3, (24, 18, 11)), (3, (64, 9, 7)), (2, (260, 37))])
def test_derived_codes_and_lane_widths_match_stored_codes(ndim, dims):
    """A plan without a mask derives the counter codes from cell coordinates;
    with an all-ones mask it reads the stored codes.  Every operator apply
    must agree bitwise between the two, and between 1, 2 and 4 cells per lane."""
    import paper_2311_16935_amd as pi

    announce("codes/lanes", dims)
    w = synth.random_small(51, ndim, dims, mask_frac=0.0)
    shape = tuple(reversed(dims))
    ones = torch.ones(shape, dtype=torch.uint8)
    gen = pi.Plan(w.dims, w.spacing, mask=None)
    stored = pi.Plan(w.dims, w.spacing, mask=ones)
    x = torch.randn(shape, device=DEV)
    for op in (pi.PI_OP_M, pi.PI_OP_N, pi.PI_OP_L):
        outs = []
        for plan in (gen, stored):
            for lanes in (1, 2, 4):
                pi.pi_set_tile(plan.handle, 3, lanes)
                assert pi.pi_get_lane_cells(plan.handle) == lanes
                outs.append(plan.apply(op, x).cpu())
        for o in outs[1:]:
            assert torch.equal(o, outs[0]), op
    # the solve reads the same codes: identical trajectories at equal tiles
    g = [t.to(DEV, torch.float32) for t in w.grads]
    sys_ = oracle_for(w)
    ref = fixed_point(sys_, sys_.source([np_(x).astype(np.float64) for x in g]))
    for lanes in (4, 2):
        pi.pi_set_tile(gen.handle, 0, lanes)
        pi.pi_set_tile(stored.handle, 0, lanes)
        a = gen.solve(g, tol=1e-9, max_iter=100000)
        b = stored.solve(g, tol=1e-9, max_iter=100000)
        assert a.info["outer_iters"] == b.info["outer_iters"]
        assert torch.equal(a.P.cpu(), b.P.cpu())
        # and it reaches the oracle's fixed point with two cells per lane too
        assert rel_maxabs(np_(a.P).astype(np.float64).ravel(), ref) <= 1e-5, lanes
    gen.close()
    stored.close()


FP_CASES = [fp64_cases()[0], fp64_cases()[2], fp64_cases()[4], fp32_cases()[1], fp32_cases()[3]]


@pytest.mark.parametrize("ndim,dims,mask_frac", [(3, (36, 13, 11), 0.1), (3, (20, 9, 17), 0.0), (2, (44, 23), 0.1)])
def test_apply_is_independent_of_segment_length(ndim, dims, mask_frac):
    """The operator apply keeps loads of planes ahead in flight and walks
    whole rounds of planes before a remainder; segment lengths from one plane
    to the whole march axis (each remainder length, ragged last segments) and
    both lane widths must give the same bits, equal to the oracle's product."""
    import paper_2311_16935_amd as pi

    announce("apply/segments", dims, mask_frac)
    w = synth.random_small(61, ndim, dims, mask_frac=mask_frac)
    sys_ = oracle_for(w)
    plan = pi.Plan(w.dims, w.spacing, mask=w.mask)
    rng = np.random.default_rng(7)
    x = np.zeros(sys_.valid.shape)
    x[sys_.valid] = rng.normal(size=sys_.n)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    xv = xt.cpu().double().numpy()[sys_.valid]
    nm = dims[-1]
    for op, mat in ((pi.PI_OP_M, sys_.M), (pi.PI_OP_N, sys_.N), (pi.PI_OP_L, sys_.L)):
        ref = mat @ xv
        first = None
        for lanes in (1, 4):
            for mseg in (1, 2, 3, 4, 5, 7, 8, nm):
                pi.pi_set_tile(plan.handle, mseg, lanes)
                y = plan.apply(op, xt).cpu()
                if first is None:
                    first = y
                    yv = y.double().numpy()
                    assert np.all(yv[~sys_.valid] == 0)
                    assert np.abs(yv[sys_.valid] - ref).max() / np.abs(ref).max() < 2e-6, op
                assert torch.equal(y, first), (op, lanes, mseg)
    plan.close()


@pytest.mark.parametrize("name,make", FP_CASES, ids=[c[0] for c in FP_CASES])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_fixed_point_cg_variant_reaches_the_same_field(name, make, fp64):
    """The PI_FIXED_POINT_CG variant solves the fixed point of Eq.
    MatrixEquation directly; its converged field must meet the same bars
    against the oracle's fixed point, in far fewer inner iterations."""
    import paper_2311_16935_amd as pi

    announce("fixed-point cg", name, fp64)
    w = make()
    sys_ = oracle_for(w)
    g = _grads(w, fp64)
    plan = pi.Plan(w.dims, w.spacing, mask=w.mask, fp64=fp64, fixed_point=True)
    res = plan.solve(g, tol=1e-13 if fp64 else 1e-10, max_iter=2000)
    assert res.status == 0, res.info
    P = np_(res.P).astype(np.float64)
    assert np.all(np.isnan(P[~sys_.valid]))
    ref = fixed_point(sys_, sys_.source([np_(x).astype(np.float64) for x in g]))
    err = rel_maxabs(P[sys_.valid], ref)
    assert err <= (1e-11 if fp64 else 1e-5), err
    # the paper's iteration needs many more passes for the same tolerance
    base = _plan(w, fp64).solve(g, tol=1e-6, max_iter=300000)
    fast = plan.solve(g, tol=1e-6, max_iter=2000)
    assert fast.info["inner_iters_total"] < base.info["inner_iters_total"]
    plan.close()


@pytest.mark.parametrize("fixed_point", [False, True], ids=["paper_iteration", "fixed_point_variant"])
@pytest.mark.parametrize("dims", [(40, 23, 17), (32, 5, 6), (256, 9, 8), (500, 9, 8), (260, 7, 9), (504, 11, 9),
                                  (752, 8, 7)],
                         ids=["interior_and_layers", "layers_only", "full_strip", "split_row", "split_row_short_tail",
                              "split_row_longest", "split_row_three_windows"])
def test_cg_passes_that_evaluate_q_again(dims, fixed_point):
    """3-D FP32 grids without missing data at four cells per lane: the CG
    passes after the first evaluate q = M p again instead of reading it
    (interior blocks and boundary-layer blocks of one kernel).  The converged
    field must match the oracle's fixed point; (32, 5, 6) has no interior
    rows or planes, so the boundary tasks do all the work; rows of 500, 260
    and 504 cells are split over two overlapping wave windows (the second
    starts at cell 244, 4 and 248 and owns the cells from 252 on; 504 is the
    longest row two windows cover); a row of 752 takes three, the middle one
    [248, 504) owning [252, 500)."""
    import paper_2311_16935_amd as pi
    from oracle.solve import fixed_point_cg

    announce("q evaluated again", dims, fixed_point)
    w = synth.random_small(83, 3, dims, anisotropic=True, mask_frac=0.0)
    g = _grads(w, False)
    plan = pi.Plan(w.dims, w.spacing, fixed_point=fixed_point)
    pi.pi_set_tile(plan.handle, 4, 4)
    assert pi.pi_get_cg_recompute(plan.handle) == 1
    res = plan.solve(g, tol=1e-9, max_iter=200000)
    assert res.status == 0, res.info
    sys_ = oracle_for(w)
    ref = fixed_point_cg(sys_, sys_.source([np_(x).astype(np.float64) for x in g]), rtol=1e-13).P
    err = rel_maxabs(np_(res.P).astype(np.float64).ravel(), ref)
    print(f"q evaluated again {dims}: outer {res.info['outer_iters']}, err {err:.2e}")
    assert err <= 1e-5, err
    # the same plan at two cells per lane stores q: same field
    pi.pi_set_tile(plan.handle, 4, 2)
    assert pi.pi_get_cg_recompute(plan.handle) == 0
    res2 = plan.solve(g, tol=1e-9, max_iter=200000)
    assert res2.status == 0, res2.info
    assert rel_maxabs(np_(res2.P).astype(np.float64).ravel(), ref) <= 1e-5
    plan.close()


@pytest.mark.parametrize("nx,expect", [(256, 1), (260, 1), (504, 1), (508, 0), (512, 0), (752, 1), (756, 0)])
def test_which_row_lengths_evaluate_q_again(nx, expect):
    """Rows split over overlapping wave windows evaluate q again only where
    the windows are as many as the plan's 256-cell strips (first window 252
    owned cells, middle ones 248, last up to 252)."""
    import paper_2311_16935_amd as pi

    plan = pi.Plan((nx, 7, 7), (1.0, 1.0, 1.0))
    pi.pi_set_tile(plan.handle, 4, 4)
    assert pi.pi_get_cg_recompute(plan.handle) == expect
    plan.close()


@pytest.mark.parametrize("fixed_point", [False, True], ids=["paper_iteration", "fixed_point_variant"])
@pytest.mark.parametrize("lanes", [1, 4])
def test_many_block_grid_takes_alpha_and_beta_from_a_finalize_kernel(fixed_point, lanes):
    """An instance of more than 1024 blocks (here 2113: 64 x 130 x 130 cells,
    one or four cells per lane (one wave per row either way), two-plane
    segments) gets the CG scalars from a finalize kernel after each pass
    instead of re-summing the partials in every block; both routes must reach
    the oracle's fixed point.  At four cells per lane the passes evaluate q
    again (two kernels per pass before the finalize)."""
    import paper_2311_16935_amd as pi
    from oracle.solve import fixed_point_cg

    announce("finalize route", fixed_point)
    w = synth.random_small(71, 3, (64, 130, 130), anisotropic=False, mask_frac=0.0)
    g = _grads(w, False)
    plan = pi.Plan(w.dims, w.spacing, fixed_point=fixed_point)
    pi.pi_set_tile(plan.handle, 2, lanes)
    assert pi.pi_get_cg_recompute(plan.handle) == (1 if lanes == 4 else 0)
    waves = 1 * 130 * 65
    assert (waves + 3) // 4 > 1024
    res = plan.solve(g, tol=1e-9, max_iter=200000)
    assert res.status == 0, res.info
    sys_ = oracle_for(w)
    ref = fixed_point_cg(sys_, sys_.source([np_(x).astype(np.float64) for x in g]), rtol=1e-13).P
    err = rel_maxabs(np_(res.P).astype(np.float64).ravel(), ref)
    print(f"finalize route: outer {res.info['outer_iters']}, inner {res.info['inner_iters_total']}, err {err:.2e}")
    assert err <= 1e-5, err
    plan.close()
