"""Time-resolved sequences (paper_2311_16935_amd.sequence): each snapshot
warm-started from the previous snapshot's pressure converges to the same
fixed point as the oracle, in fewer outer steps than from zero."""

import numpy as np
import pytest
import torch

from gpu_common import DEV, announce, requires_gpu
from oracle.solve import fixed_point
from oracle.system import assemble

pytestmark = [pytest.mark.gpu, requires_gpu]


def _rel_maxabs(a, b):
    return float(np.abs(a - b).max() / np.sqrt(np.mean(b ** 2)))


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_drifting_blobs_sequence(fp64):
    import paper_2311_16935_amd as pi
    import synth
    from paper_2311_16935_amd.sequence import solve_sequence

    announce("sequence drifting blobs", "fp64" if fp64 else "fp32")
    dims = (28, 24, 20)
    dt = torch.float64 if fp64 else torch.float32
    snaps = []
    for k in range(4):
        _, g, sp = synth.gaussian_blobs(dims, seed=77, nblobs=12, sigma_range=(0.08, 0.2), with_pressure=False,
                                        t=float(k), speed=0.015)
        snaps.append([c.to(dt).to(DEV).contiguous() for c in g])
    plan = pi.Plan(dims, sp, fp64=fp64)
    tol = 1e-14 if fp64 else 1e-9
    cold = solve_sequence(plan, snaps, tol=tol, max_iter=300000, warm=False)
    warm = solve_sequence(plan, snaps, tol=tol, max_iter=300000, warm=True)
    sys_ = assemble(np.ones(tuple(reversed(dims)), np.uint8), sp)
    for k, (c, w) in enumerate(zip(cold, warm)):
        for r in (c, w):
            assert r.status == 0 or (fp64 and r.status == pi.PI_ERR_NOT_CONVERGED and r.info["eps_R"] <= 1e-13), r.info
        ref = fixed_point(sys_, sys_.source([x.cpu().numpy().astype(np.float64) for x in snaps[k]]))
        err = _rel_maxabs(sys_.from_grid(w.P.cpu().numpy().astype(np.float64)), ref)
        assert err <= (1e-11 if fp64 else 1e-5), (k, err)
        if k > 0:
            assert w.info["outer_iters"] < c.info["outer_iters"], (k, w.info, c.info)
    plan.close()


def test_taylor_vortex_sequence_from_velocity():
    """The paper's Taylor-vortex series (26 snapshots, 0.05 <= t <= 0.3,
    101^2 on [-3, 3]^2): velocity -> source -> pressure, warm-started from
    the previous snapshot; the same answers as cold solves, fewer outer
    steps in total."""
    import paper_2311_16935_amd as pi
    import synth
    from paper_2311_16935_amd import flow
    from paper_2311_16935_amd.sequence import solve_sequence

    announce("sequence taylor vortex")
    n, dtv = 101, 1e-4
    srcs = []
    for t in np.linspace(0.05, 0.3, 26):
        u, _, sp = synth.taylor_velocity((n, n), t=t)
        up = synth.taylor_velocity((n, n), t=t - dtv)[0]
        un = synth.taylor_velocity((n, n), t=t + dtv)[0]
        dev = [[c.float().to(DEV).contiguous() for c in v] for v in (u, up, un)]
        srcs.append(flow.pi_flow_source(flow.PI_FLOW_NS, dev[0], sp, u_prev=dev[1], u_next=dev[2], rho=1.0, mu=1.0,
                                        dt=dtv))
    plan = pi.Plan((n, n), sp)
    cold = solve_sequence(plan, srcs, tol=1e-7, warm=False)
    warm = solve_sequence(plan, srcs, tol=1e-7, warm=True)
    for c, w in zip(cold, warm):
        assert c.status == 0 and w.status == 0
        scale = float(c.P.abs().max())
        assert float((c.P - w.P).abs().max()) <= 1e-4 * scale
    assert sum(w.info["outer_iters"] for w in warm) < sum(c.info["outer_iters"] for c in cold)
    plan.close()
