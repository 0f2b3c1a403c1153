"""The 2-D cell-centred scheme (PI_CELL_CENTERED) through the C interface
against the cell-centred oracle (oracle/cellcentered.py): the three
operators and the source on masked, ragged and degenerate grids, solves in
FP64 (1e-11 of RMS(P)) and FP32 (1e-5) of the paper's iteration and of the
fixed-point CG variant, the gauge over diagonally connected groups, and
exact recovery of a quadratic pressure field."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, announce, np_, rel_maxabs, requires_gpu
from oracle.cellcentered import assemble_cc
from oracle.solve import fixed_point, gauge

pytestmark = [pytest.mark.gpu, requires_gpu]


def _oracle(w):
    mask = np.ones(tuple(reversed(w.dims)), np.uint8) if w.mask is None else np_(w.mask)
    return assemble_cc(mask, w.spacing)


def _plan(w, fp64, **kw):
    import paper_2311_16935_amd as pi

    return pi.Plan(w.dims, w.spacing, mask=w.mask, fp64=fp64, cell_centered=True, **kw)


def _grads(w, fp64):
    dt = torch.float64 if fp64 else torch.float32
    return [g.to(dt).to(DEV).contiguous() for g in w.grads]


CASES = [
    ("masked_45x37", lambda: synth.random_small(41, 2, (45, 37), mask_frac=0.1)),
    ("iso_unmasked_64x48", lambda: synth.random_small(12, 2, (64, 48), anisotropic=False, mask_frac=0.0)),
    ("masked_197x131", lambda: synth.random_small(11, 2, (197, 131), mask_frac=0.1)),
    ("masked_96x45", lambda: synth.random_small(21, 2, (96, 45), mask_frac=0.1)),   # four cells per lane
    ("masked_520x36", lambda: synth.random_small(22, 2, (520, 36), mask_frac=0.1)),  # several strips
    ("thin_1x23", lambda: synth.random_small(17, 2, (1, 23), mask_frac=0.0)),
    ("thin_2x19", lambda: synth.random_small(18, 2, (2, 19), mask_frac=0.0)),
    ("thin_31x3", lambda: synth.random_small(19, 2, (31, 3), mask_frac=0.1)),
]


def _converged_fp64(res):
    return res.status == 0 or (res.status == 4 and res.info["eps_R"] <= 1e-13)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_operators_and_source_match_the_oracle(name, make):
    import paper_2311_16935_amd as pi

    announce("cc operators", name)
    w = make()
    s = _oracle(w)
    rng = np.random.default_rng(5)
    for fp64, bar in ((True, 1e-13), (False, 2e-6)):
        plan = _plan(w, fp64)
        dt = torch.float64 if fp64 else torch.float32
        x = torch.from_numpy(rng.normal(size=plan.shape)).to(dt).to(DEV)
        xv = s.from_grid(np_(x).astype(np.float64))
        for op, A in ((pi.PI_OP_M, s.M), (pi.PI_OP_N, s.N), (pi.PI_OP_L, s.L)):
            y = plan.apply(op, x)
            ref = A @ xv
            got = s.from_grid(np_(y).astype(np.float64))
            assert np.abs(got - ref).max() <= bar * np.abs(xv).max() * 4, (name, op, fp64)
            assert np.all(np_(y)[~s.valid] == 0)
        S = plan.source(_grads(w, fp64))
        ref = s.source([np_(g).astype(np.float64) for g in _grads(w, fp64)])
        got = s.from_grid(np_(S).astype(np.float64))
        assert np.abs(got - ref).max() <= bar * np.abs(ref).max() * 4, (name, "source", fp64)
        plan.close()


# grids whose fixed point FP64 resolves to 1e-11 of RMS(P)
FP64_CASES = [c for c in CASES if c[0] not in ("masked_197x131", "masked_520x36")]


@pytest.mark.parametrize("name,make", FP64_CASES, ids=[c[0] for c in FP64_CASES])
@pytest.mark.parametrize("fixed_point_cg", [False, True], ids=["paper", "variant"])
def test_solve_fp64_matches_fixed_point(name, make, fixed_point_cg):
    announce("cc solve fp64", name, fixed_point_cg)
    w = make()
    s = _oracle(w)
    plan = _plan(w, True, fixed_point=fixed_point_cg)
    g = _grads(w, True)
    res = plan.solve(g, tol=1e-14, max_iter=300000, check=False)
    assert _converged_fp64(res), res.info
    P = np_(res.P)
    assert np.all(np.isnan(P[~s.valid]))
    ref = fixed_point(s, s.source([np_(x) for x in g]))
    err = rel_maxabs(P[s.valid], ref)
    assert err <= 1e-11, (err, res.info)
    plan.close()


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fixed_point_cg", [False, True], ids=["paper", "variant"])
def test_solve_fp32_matches_fixed_point(name, make, fixed_point_cg):
    announce("cc solve fp32", name, fixed_point_cg)
    w = make()
    s = _oracle(w)
    plan = _plan(w, False, fixed_point=fixed_point_cg)
    g = _grads(w, False)
    res = plan.solve(g, tol=1e-10, max_iter=300000)
    assert res.status == 0, res.info
    ref = fixed_point(s, s.source([np_(x).astype(np.float64) for x in g]))
    assert rel_maxabs(np_(res.P).astype(np.float64)[s.valid], ref) <= 1e-5
    plan.close()


def test_gauge_counts_diagonal_neighbours():
    """Two blocks of data that touch only at a corner form one group in the
    cell-centred scheme (a diagonal ray joins them), two in the face-crossing
    one."""
    import paper_2311_16935_amd as pi

    announce("cc diagonal group")
    ny, nx = 12, 14
    m = np.zeros((ny, nx), np.uint8)
    m[:6, :7] = 1
    m[6:, 7:] = 1
    rng = np.random.default_rng(2)
    g = [torch.from_numpy(np.where(m == 1, rng.normal(size=m.shape), np.nan)).to(DEV) for _ in range(2)]
    sp = (1.0, 0.8)
    s = assemble_cc(m, sp)
    plan = pi.Plan((nx, ny), sp, mask=m, fp64=True, cell_centered=True)
    res = plan.solve(g, tol=1e-14, max_iter=300000, check=False)
    assert _converged_fp64(res), res.info
    assert res.info["components"] == 1
    ref = fixed_point(s, s.source([np_(x) for x in g]))
    assert rel_maxabs(np_(res.P)[s.valid], ref) <= 1e-11
    plan.close()
    fc = pi.Plan((nx, ny), sp, mask=m, fp64=True)
    assert fc.solve(g, tol=1e-8).info["components"] == 2
    fc.close()


def test_quadratic_pressure_is_recovered_exactly():
    import paper_2311_16935_amd as pi

    announce("cc quadratic")
    P, g, sp = synth.quadratic((53, 41), seed=4)
    m = np_(synth.disk_mask((53, 41), seed=4, frac=0.08))
    Pm = np.where(m == 1, np_(P), np.nan)
    gg = [torch.from_numpy(np.where(m == 1, np_(c), np.nan)).to(DEV) for c in g]
    plan = pi.Plan((53, 41), sp, mask=m, fp64=True, cell_centered=True)
    res = plan.solve(gg, tol=1e-13, max_iter=300000, check=False)
    assert _converged_fp64(res) or res.info["eps_R"] <= 1e-12, res.info
    s = assemble_cc(m, sp)
    want = gauge(s, s.from_grid(Pm))
    got = np_(res.P)[s.valid]
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    plan.close()


def test_mixed_batch_of_schemes_and_shapes():
    """One batched call over cell-centred plans (one and four cells per lane)
    and face-crossing 2-D and 3-D plans: every instance matches its own
    oracle's fixed point."""
    import paper_2311_16935_amd as pi
    from oracle.system import assemble

    announce("cc mixed batch")
    specs = [(synth.random_small(31, 2, (45, 37), mask_frac=0.1), True),
             (synth.random_small(32, 2, (96, 45), mask_frac=0.1), True),
             (synth.random_small(33, 2, (60, 41), mask_frac=0.1), False),
             (synth.random_small(34, 3, (24, 17, 13), mask_frac=0.1), False)]
    plans, grads, refs = [], [], []
    for w, cc in specs:
        mask = np.ones(tuple(reversed(w.dims)), np.uint8) if w.mask is None else np_(w.mask)
        s = assemble_cc(mask, w.spacing) if cc else assemble(mask, w.spacing)
        g = _grads(w, False)
        plans.append(pi.Plan(w.dims, w.spacing, mask=w.mask, cell_centered=cc))
        grads.append(g)
        refs.append((s, fixed_point(s, s.source([np_(x).astype(np.float64) for x in g]))))
    rc, Ps, infos = pi.solve_batched(plans, grads, tol=1e-10, max_iter=300000)
    assert rc == 0, infos
    for (s, ref), P, info in zip(refs, Ps, infos):
        assert info["status"] == 0, info
        assert rel_maxabs(np_(P).astype(np.float64)[s.valid], ref) <= 1e-5
    for p in plans:
        p.close()
