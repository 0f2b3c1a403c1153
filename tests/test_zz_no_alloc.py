"""pi_solve_batched_noalloc against pi_solve_batched, through the C interface.

The no-allocation entry point runs the batched solve's kernels with its
per-call buffers in the library's static scratch array.  Two calls in a row
(the second with fewer, smaller grids, so stale contents of the array from
the first would show) must return what pi_solve_batched returns: the same
status and outer-step counts, the same fields (the reductions are fixed-order,
so bit for bit), and fields within 1e-5 RMS(P) of the oracle's fixed point.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, announce, np_, oracle_for, rel_maxabs, requires_gpu
from oracle.solve import fixed_point

pytestmark = [pytest.mark.gpu, requires_gpu]


def _batch(cases):
    import paper_2311_16935_amd as pi

    works = [make() for make in cases]
    plans = [pi.Plan(w.dims, w.spacing, mask=w.mask) for w in works]
    grads = [[g.to(DEV, torch.float32) for g in w.grads] for w in works]
    return works, plans, grads


def _run(pi, plans, grads, noalloc):
    P = [torch.full(p.shape, 7.0, dtype=torch.float32, device=DEV) for p in plans]
    rc, P, infos = pi.solve_batched(plans, grads, P, tol=1e-9, max_iter=200000, noalloc=noalloc)
    return rc, P, infos


def test_noalloc_matches_batched_on_two_calls():
    import paper_2311_16935_amd as pi

    first = [lambda: synth.random_small(61, 2, (197, 131), mask_frac=0.1),
             lambda: synth.random_small(62, 3, (48, 24, 20), mask_frac=0.0),
             lambda: synth.random_small(63, 3, (33, 65, 17), anisotropic=False, mask_frac=0.1),
             lambda: synth.random_small(64, 2, (132, 90), mask_frac=0.0)]
    second = [lambda: synth.random_small(65, 2, (45, 37), mask_frac=0.1),
              lambda: synth.random_small(66, 3, (24, 17, 13), mask_frac=0.0)]
    for call, cases in enumerate((first, second)):
        announce("noalloc batched call", call, len(cases))
        works, plans, grads = _batch(cases)
        rc_a, P_a, inf_a = _run(pi, plans, grads, noalloc=False)
        rc_b, P_b, inf_b = _run(pi, plans, grads, noalloc=True)
        assert rc_a == pi.PI_OK and rc_b == pi.PI_OK, (rc_a, rc_b)
        for k, (w, a, b, ia, ib) in enumerate(zip(works, P_a, P_b, inf_a, inf_b)):
            assert ia["status"] == ib["status"] == 0
            assert ia["outer_iters"] == ib["outer_iters"]
            assert ia["inner_iters_total"] == ib["inner_iters_total"]
            assert torch.equal(torch.nan_to_num(a, 123.0), torch.nan_to_num(b, 123.0)), w.name
            sys_ = oracle_for(w)
            ref = fixed_point(sys_, sys_.source([np_(x).astype(np.float64) for x in grads[k]]))
            got = np_(b).astype(np.float64)[sys_.valid]
            assert rel_maxabs(got, ref) <= 1e-5, w.name
        for p in plans:
            p.close()


def test_noalloc_rejects_more_instances_than_its_scratch_holds():
    import paper_2311_16935_amd as pi

    n = pi.PI_NOALLOC_MAX_INSTANCES + 1
    w = synth.random_small(67, 2, (8, 8), mask_frac=0.0)
    plan = pi.Plan(w.dims, w.spacing)
    g = [x.to(DEV, torch.float32) for x in w.grads]
    P = torch.zeros(plan.shape, dtype=torch.float32, device=DEV)
    rc, _ = pi.pi_solve_batched_noalloc([plan.handle] * n, [g[0]] * n, [g[1]] * n, None, [P] * n, [1e-6] * n, 10)
    assert rc == pi.PI_ERR_TOO_LARGE
    plan.close()
